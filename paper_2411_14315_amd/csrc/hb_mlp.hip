// Learned Newton warm start: a small multilayer perceptron (BF16 weights,
// FP32 accumulation) with hand-written forward, backward and Adam kernels,
// and the POD expansion Y = mean + sum_k c_k phi_k that turns its output
// into a modal initial guess for hb_newton_solve.
//
// Parameter layout (also the gradient layout): for each layer l,
// W_l [out_l][in_l] row-major followed by b_l [out_l].  Hidden layers use
// ReLU; the last layer is linear.  The loss is the mean squared error
// (1 / (B out)) sum (y - t)^2.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "hb.h"
#include "hb_internal.h"

namespace {

constexpr int BLK = 256;

int mfail(int code, const std::string& msg) {
  hb::set_last_error(msg);
  return code;
}

#define HB_MCHECK(...)                                                              \
  do {                                                                              \
    hipError_t e_ = (__VA_ARGS__);                                                  \
    if (e_ != hipSuccess)                                                           \
      return mfail(e_ == hipErrorOutOfMemory ? HB_ERR_OOM : HB_ERR_DEVICE,          \
                   std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_));       \
  } while (0)

// round-to-nearest-even FP32 -> BF16 (NaN kept quiet), and back
__host__ __device__ inline uint16_t to_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float from_bf16(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

// Z[b][o] = b_o + sum_i W[o][i] X[b][i];  A = relu(Z) (or Z for the last layer)
__global__ void __launch_bounds__(BLK)
k_dense_fwd(const float* __restrict__ X, const uint16_t* __restrict__ W,
            const uint16_t* __restrict__ bias, int B, int in, int out, int relu,
            float* __restrict__ Z, float* __restrict__ A) {
  const int gid = blockIdx.x * BLK + threadIdx.x;
  if (gid >= B * out) return;
  const int b = gid / out, o = gid - b * out;
  float z = from_bf16(bias[o]);
  const float* x = X + (size_t)b * in;
  const uint16_t* w = W + (size_t)o * in;
  for (int i = 0; i < in; ++i) z += from_bf16(w[i]) * x[i];
  Z[gid] = z;
  A[gid] = relu ? fmaxf(z, 0.0f) : z;
}

__global__ void k_zero1(double* x) { *x = 0.0; }

// dY = 2 (Y - T) / (B out); loss partial sums in FP64
__global__ void __launch_bounds__(BLK)
k_mse_grad(const float* __restrict__ Y, const float* __restrict__ T, int n, float scale,
           float* __restrict__ dY, double* __restrict__ loss) {
  __shared__ double red[BLK / 64];
  const int gid = blockIdx.x * BLK + threadIdx.x;
  double l = 0.0;
  if (gid < n) {
    const float d = Y[gid] - T[gid];
    dY[gid] = 2.0f * d * scale;
    l = (double)d * (double)d * (double)scale;
  }
  for (int o = 32; o > 0; o >>= 1) l += __shfl_down(l, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < BLK / 64; ++q) t += red[q];
    atomicAdd(loss, t);
  }
}

// gW[o][i] = sum_b dZ[b][o] X[b][i]; gb[o] = sum_b dZ[b][o]
__global__ void __launch_bounds__(BLK)
k_dense_bwd_w(const float* __restrict__ dZ, const float* __restrict__ X, int B, int in, int out,
              float* __restrict__ gW, float* __restrict__ gb) {
  const int gid = blockIdx.x * BLK + threadIdx.x;
  if (gid >= out * (in + 1)) return;
  const int o = gid / (in + 1), i = gid - o * (in + 1);
  float s = 0.0f;
  if (i < in) {
    for (int b = 0; b < B; ++b) s += dZ[(size_t)b * out + o] * X[(size_t)b * in + i];
    gW[(size_t)o * in + i] = s;
  } else {
    for (int b = 0; b < B; ++b) s += dZ[(size_t)b * out + o];
    gb[o] = s;
  }
}

// dX[b][i] = (sum_o W[o][i] dZ[b][o]) * relu'(Zprev[b][i])
__global__ void __launch_bounds__(BLK)
k_dense_bwd_x(const float* __restrict__ dZ, const uint16_t* __restrict__ W,
              const float* __restrict__ Zprev, int B, int in, int out, float* __restrict__ dX) {
  const int gid = blockIdx.x * BLK + threadIdx.x;
  if (gid >= B * in) return;
  const int b = gid / in, i = gid - b * in;
  float s = 0.0f;
  for (int o = 0; o < out; ++o) s += from_bf16(W[(size_t)o * in + i]) * dZ[(size_t)b * out + o];
  dX[gid] = Zprev[gid] > 0.0f ? s : 0.0f;
}

// Adam with bias correction on the FP32 master copy; refresh the BF16 copy.
__global__ void __launch_bounds__(BLK)
k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
       const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps,
       float c1, float c2, uint16_t* __restrict__ w16) {
  const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  w16[i] = to_bf16(wi);
}

// Y[i] = base[i] + mean[i] + sum_k c_k basis[k][i]   (base optional)
__global__ void __launch_bounds__(BLK)
k_pod_expand(int64_t L, int r, const double* base, const double* __restrict__ mean,
             const double* __restrict__ basis, const float* __restrict__ coef, double* Y) {
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < L; i += stride) {
    double y = base ? base[i] + mean[i] : mean[i];
    for (int k = 0; k < r; ++k) y += (double)coef[k] * basis[(int64_t)k * L + i];
    Y[i] = y;
  }
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + BLK - 1) / BLK); }

// Device-resident activation storage of hb_mlp_forward_noalloc: one copy per
// GPU, held until the process ends.  In host code `scratch` only names the
// symbol; its device address comes from hipGetSymbolAddress (per device).
constexpr int64_t kScratchFloats = int64_t(4) << 20;  // 16 MiB
__device__ __align__(256) float scratch[kScratchFloats];
constexpr int kMaxDevices = 64;
float* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// The address of this device's `scratch` (looked up once per device).
hipError_t scratch_ptr(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
  hipError_t ensure(size_t b) {
    if (p && b <= bytes) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    hipError_t e = hipMalloc(&p, b ? b : 8);
    bytes = e == hipSuccess ? b : 0;
    return e;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

}  // namespace

struct hb_mlp {
  std::vector<int32_t> widths;
  std::vector<int64_t> woff, boff;  // parameter offsets of W_l and b_l
  int64_t nparam = 0;
  Buf master, w16, m1, m2, grad, loss;
  Buf act;  // per layer Z and A for the last batch: sizes grow with B
  int64_t act_B = 0;
  std::vector<int64_t> zoff, aoff;
  Buf dbuf0, dbuf1;  // backward scratch [B][max width]
  int64_t step = 0;
  int layers() const { return (int)widths.size() - 1; }
};

namespace {

int ensure_batch(hb_mlp* n, int B) {
  if (B <= n->act_B) return HB_OK;
  int64_t off = 0;
  n->zoff.assign(n->layers() + 1, 0);
  n->aoff.assign(n->layers() + 1, 0);
  for (int l = 1; l <= n->layers(); ++l) {
    n->zoff[l] = off;
    off += (int64_t)B * n->widths[l];
    n->aoff[l] = off;
    off += (int64_t)B * n->widths[l];
  }
  int maxw = 0;
  for (int w : n->widths) maxw = w > maxw ? w : maxw;
  HB_MCHECK(n->act.ensure(sizeof(float) * off));
  HB_MCHECK(n->dbuf0.ensure(sizeof(float) * (size_t)B * maxw));
  HB_MCHECK(n->dbuf1.ensure(sizeof(float) * (size_t)B * maxw));
  n->act_B = B;
  return HB_OK;
}

int forward(hb_mlp* n, const float* X, int B, hipStream_t st) {
  int rc = ensure_batch(n, B);
  if (rc) return rc;
  float* act = n->act.as<float>();
  const uint16_t* w16 = n->w16.as<uint16_t>();
  const float* in = X;
  for (int l = 1; l <= n->layers(); ++l) {
    const int ni = n->widths[l - 1], no = n->widths[l];
    float* Z = act + n->zoff[l];
    float* A = act + n->aoff[l];
    hipLaunchKernelGGL(k_dense_fwd, dim3(nblocks((int64_t)B * no)), dim3(BLK), 0, st, in,
                       w16 + n->woff[l - 1], w16 + n->boff[l - 1], B, ni, no,
                       l < n->layers() ? 1 : 0, Z, A);
    HB_MCHECK(hipGetLastError());
    in = A;
  }
  return HB_OK;
}

}  // namespace

extern "C" {

int hb_mlp_create(int32_t n_layers, const int32_t* widths, const float* params, uint64_t seed,
                  hb_mlp** out) {
  if (!out || !widths || n_layers < 1 || n_layers > 16) return mfail(HB_ERR_ARG, "bad layers");
  *out = nullptr;
  std::unique_ptr<hb_mlp> n(new hb_mlp());
  for (int l = 0; l <= n_layers; ++l) {
    if (widths[l] < 1 || widths[l] > 4096) return mfail(HB_ERR_ARG, "width out of range");
    n->widths.push_back(widths[l]);
  }
  for (int l = 0; l < n_layers; ++l) {
    n->woff.push_back(n->nparam);
    n->nparam += (int64_t)widths[l] * widths[l + 1];
    n->boff.push_back(n->nparam);
    n->nparam += widths[l + 1];
  }
  std::vector<float> p(n->nparam, 0.0f);
  if (params) {
    for (int64_t i = 0; i < n->nparam; ++i) {
      if (!std::isfinite(params[i])) return mfail(HB_ERR_ARG, "non-finite parameter");
      p[i] = params[i];
    }
  } else {
    // He-uniform weights from a 64-bit linear congruential stream; zero biases
    uint64_t s = seed * 6364136223846793005ull + 1442695040888963407ull;
    for (int l = 0; l < n_layers; ++l) {
      const float a = std::sqrt(6.0f / (float)widths[l]);
      for (int64_t i = 0; i < (int64_t)widths[l] * widths[l + 1]; ++i) {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        const float u = (float)((s >> 11) * (1.0 / 9007199254740992.0));
        p[n->woff[l] + i] = a * (2.0f * u - 1.0f);
      }
    }
  }
  std::vector<uint16_t> p16(n->nparam);
  for (int64_t i = 0; i < n->nparam; ++i) {
    p16[i] = to_bf16(p[i]);
    p[i] = from_bf16(p16[i]);  // the master starts at the representable value
  }
  HB_MCHECK(n->master.ensure(sizeof(float) * n->nparam));
  HB_MCHECK(n->w16.ensure(sizeof(uint16_t) * n->nparam));
  HB_MCHECK(n->m1.ensure(sizeof(float) * n->nparam));
  HB_MCHECK(n->m2.ensure(sizeof(float) * n->nparam));
  HB_MCHECK(n->grad.ensure(sizeof(float) * n->nparam));
  HB_MCHECK(n->loss.ensure(sizeof(double)));
  HB_MCHECK(hipMemcpy(n->master.p, p.data(), sizeof(float) * n->nparam, hipMemcpyHostToDevice));
  HB_MCHECK(hipMemcpy(n->w16.p, p16.data(), sizeof(uint16_t) * n->nparam, hipMemcpyHostToDevice));
  HB_MCHECK(hipMemset(n->m1.p, 0, sizeof(float) * n->nparam));
  HB_MCHECK(hipMemset(n->m2.p, 0, sizeof(float) * n->nparam));
  *out = n.release();
  return HB_OK;
}

void hb_mlp_destroy(hb_mlp* n) { delete n; }

int hb_mlp_num_params(const hb_mlp* n, int64_t* count) {
  if (!n || !count) return mfail(HB_ERR_ARG, "NULL argument");
  *count = n->nparam;
  return HB_OK;
}

int hb_mlp_get_params(const hb_mlp* n, float* host_out) {
  if (!n || !host_out) return mfail(HB_ERR_ARG, "NULL argument");
  std::vector<uint16_t> p16(n->nparam);
  HB_MCHECK(hipMemcpy(p16.data(), n->w16.p, sizeof(uint16_t) * n->nparam, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n->nparam; ++i) host_out[i] = from_bf16(p16[i]);
  return HB_OK;
}

int hb_mlp_forward(hb_mlp* n, const float* X, int32_t B, float* Y, void* stream) {
  if (!n || !X || !Y || B < 1) return mfail(HB_ERR_ARG, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  int rc = forward(n, X, B, st);
  if (rc) return rc;
  const int L = n->layers();
  HB_MCHECK(hipMemcpyAsync(Y, n->act.as<float>() + n->aoff[L],
                           sizeof(float) * (size_t)B * n->widths[L], hipMemcpyDeviceToDevice, st));
  return HB_OK;
}

int hb_mlp_forward_noalloc(const hb_mlp* n, const float* X, int32_t B, float* Y, void* stream) {
  if (!n || !X || !Y || B < 1) return mfail(HB_ERR_ARG, "bad argument");
  int maxw = 0;
  for (int l = 1; l < n->layers(); ++l) maxw = n->widths[l] > maxw ? n->widths[l] : maxw;
  maxw = n->widths.back() > maxw ? n->widths.back() : maxw;
  // [Z | A] for two hidden layers in turn; the last layer writes A into Y
  if ((int64_t)B * maxw * 4 > kScratchFloats)
    return mfail(HB_ERR_ARG, "batch too large for the device scratch: B * max width must be <= " +
                                 std::to_string(kScratchFloats / 4));
  float* sc = nullptr;
  HB_MCHECK(scratch_ptr(&sc));
  hipStream_t st = (hipStream_t)stream;
  const uint16_t* w16 = n->w16.as<uint16_t>();
  const int64_t region = (int64_t)B * maxw;
  const float* in = X;
  for (int l = 1; l <= n->layers(); ++l) {
    const int ni = n->widths[l - 1], no = n->widths[l];
    const bool last = l == n->layers();
    float* Z = sc + (int64_t)((l - 1) & 1) * 2 * region;
    float* A = last ? Y : Z + region;
    hipLaunchKernelGGL(k_dense_fwd, dim3(nblocks((int64_t)B * no)), dim3(BLK), 0, st, in,
                       w16 + n->woff[l - 1], w16 + n->boff[l - 1], B, ni, no, last ? 0 : 1, Z,
                       A);
    HB_MCHECK(hipGetLastError());
    in = A;
  }
  return HB_OK;
}

int hb_mlp_loss_grad(hb_mlp* n, const float* X, const float* T, int32_t B, float* grad,
                     double* loss, void* stream) {
  if (!n || !X || !T || B < 1) return mfail(HB_ERR_ARG, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  int rc = forward(n, X, B, st);
  if (rc) return rc;
  const int L = n->layers();
  float* act = n->act.as<float>();
  float* g = grad ? grad : n->grad.as<float>();
  const uint16_t* w16 = n->w16.as<uint16_t>();
  float* dcur = n->dbuf0.as<float>();
  float* dnext = n->dbuf1.as<float>();
  const int no = n->widths[L];
  hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, st, n->loss.as<double>());
  hipLaunchKernelGGL(k_mse_grad, dim3(nblocks((int64_t)B * no)), dim3(BLK), 0, st,
                     act + n->aoff[L], T, B * no, 1.0f / (float)(B * no), dcur,
                     n->loss.as<double>());
  HB_MCHECK(hipGetLastError());
  for (int l = L; l >= 1; --l) {
    const int ni = n->widths[l - 1], nol = n->widths[l];
    const float* Xin = l > 1 ? act + n->aoff[l - 1] : X;
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(nblocks((int64_t)nol * (ni + 1))), dim3(BLK), 0, st,
                       dcur, Xin, B, ni, nol, g + n->woff[l - 1], g + n->boff[l - 1]);
    HB_MCHECK(hipGetLastError());
    if (l > 1) {
      hipLaunchKernelGGL(k_dense_bwd_x, dim3(nblocks((int64_t)B * ni)), dim3(BLK), 0, st, dcur,
                         w16 + n->woff[l - 1], act + n->zoff[l - 1], B, ni, nol, dnext);
      HB_MCHECK(hipGetLastError());
      float* t = dcur;
      dcur = dnext;
      dnext = t;
    }
  }
  if (loss) {
    HB_MCHECK(hipMemcpyAsync(loss, n->loss.p, sizeof(double), hipMemcpyDeviceToHost, st));
    HB_MCHECK(hipStreamSynchronize(st));
  }
  return HB_OK;
}

int hb_mlp_adam_step(hb_mlp* n, const float* grad, float lr, void* stream) {
  if (!n || !(lr > 0)) return mfail(HB_ERR_ARG, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  ++n->step;
  const float c1 = 1.0f - std::pow(b1, (float)n->step);
  const float c2 = 1.0f - std::pow(b2, (float)n->step);
  hipLaunchKernelGGL(k_adam, dim3(nblocks(n->nparam)), dim3(BLK), 0, st, n->master.as<float>(),
                     n->m1.as<float>(), n->m2.as<float>(), grad ? grad : n->grad.as<float>(),
                     n->nparam, lr, b1, b2, eps, c1, c2, n->w16.as<uint16_t>());
  HB_MCHECK(hipGetLastError());
  return HB_OK;
}

int hb_pod_expand(int64_t L, int32_t r, const double* base, const double* mean,
                  const double* basis, const float* coef, double* Y, void* stream) {
  if (L < 1 || r < 0 || !mean || (r > 0 && (!basis || !coef)) || !Y)
    return mfail(HB_ERR_ARG, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  const int64_t nb = (L + BLK - 1) / BLK;
  hipLaunchKernelGGL(k_pod_expand, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(BLK), 0, st, L, r,
                     base, mean, basis, coef, Y);
  HB_MCHECK(hipGetLastError());
  return HB_OK;
}

}  // extern "C"
