// Proper orthogonal decomposition by the method of snapshots, for the
// learned warm start's regression targets: the snapshot mean, the Gram
// matrix of the centred snapshots and the modes are formed on the device;
// the small symmetric eigenproblem of the Gram matrix is solved on the host
// (Householder tridiagonalisation, then implicit-shift QR with Wilkinson
// shifts, as in Golub and Van Loan, Matrix Computations, ch. 8).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <numeric>
#include <string>
#include <vector>

#include "hb.h"
#include "hb_internal.h"

namespace {

constexpr int BLK = 256;
constexpr int GT = 64;  // rows (and columns) of one Gram tile
constexpr int GK = 16;  // snapshot entries per LDS stage
constexpr int BR = 16;  // modes per lane of the mode kernel

int pfail(int code, const std::string& msg) {
  hb::set_last_error(msg);
  return code;
}

#define HB_PCHECK(...)                                                              \
  do {                                                                              \
    hipError_t e_ = (__VA_ARGS__);                                                  \
    if (e_ != hipSuccess)                                                           \
      return pfail(e_ == hipErrorOutOfMemory ? HB_ERR_OOM : HB_ERR_DEVICE,          \
                   std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_));       \
  } while (0)

// ------------------------------------------------------------ host eigensolver

// Householder reduction of the symmetric n x n matrix a (row-major,
// overwritten) to T = Q^T a Q; d = diag(T), e[i] = T[i][i+1], qt = Q^T.
void tridiagonalise(int n, std::vector<double>& a, std::vector<double>& d,
                    std::vector<double>& e, std::vector<double>& qt) {
  qt.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) qt[(size_t)i * n + i] = 1.0;
  std::vector<double> v(n), p(n), w(n), u(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // x = a[k+1 .. n-1][k]
    double nx = 0.0;
    for (int i = 0; i < m; ++i) {
      const double x = a[(size_t)(k + 1 + i) * n + k];
      nx += x * x;
    }
    nx = std::sqrt(nx);
    if (nx == 0.0) continue;
    const double x0 = a[(size_t)(k + 1) * n + k];
    const double alpha = x0 >= 0.0 ? -nx : nx;
    for (int i = 0; i < m; ++i) v[i] = a[(size_t)(k + 1 + i) * n + k];
    v[0] -= alpha;
    double vv = 0.0;
    for (int i = 0; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    // trailing block B <- P B P with P = I - beta v v^T
    for (int i = 0; i < m; ++i) {
      const double* row = &a[(size_t)(k + 1 + i) * n + k + 1];
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      p[i] = beta * s;
    }
    double pv = 0.0;
    for (int i = 0; i < m; ++i) pv += p[i] * v[i];
    const double half = 0.5 * beta * pv;
    for (int i = 0; i < m; ++i) w[i] = p[i] - half * v[i];
    for (int i = 0; i < m; ++i) {
      double* row = &a[(size_t)(k + 1 + i) * n + k + 1];
      for (int j = 0; j < m; ++j) row[j] -= v[i] * w[j] + w[i] * v[j];
    }
    a[(size_t)(k + 1) * n + k] = alpha;
    a[(size_t)k * n + k + 1] = alpha;
    for (int i = 1; i < m; ++i) {
      a[(size_t)(k + 1 + i) * n + k] = 0.0;
      a[(size_t)k * n + k + 1 + i] = 0.0;
    }
    // Q <- Q P, i.e. rows k+1.. of Q^T <- P (rows k+1.. of Q^T)
    std::fill(u.begin(), u.end(), 0.0);
    for (int i = 0; i < m; ++i) {
      const double* row = &qt[(size_t)(k + 1 + i) * n];
      for (int j = 0; j < n; ++j) u[j] += v[i] * row[j];
    }
    for (int i = 0; i < m; ++i) {
      double* row = &qt[(size_t)(k + 1 + i) * n];
      const double f = beta * v[i];
      for (int j = 0; j < n; ++j) row[j] -= f * u[j];
    }
  }
  d.resize(n);
  e.assign(n > 1 ? n - 1 : 0, 0.0);
  for (int i = 0; i < n; ++i) d[i] = a[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = a[(size_t)i * n + i + 1];
}

// Implicit symmetric QR steps with Wilkinson shifts on the tridiagonal
// (d, e) until every off-diagonal entry is negligible; the Givens rotations
// are applied to the rows of qt, so that row k of qt ends as the
// eigenvector of d[k].  False if 30 n steps do not suffice.
bool tridiagonal_qr(int n, std::vector<double>& d, std::vector<double>& e,
                    std::vector<double>& qt) {
  const double eps = std::numeric_limits<double>::epsilon();
  auto small = [&](int i) { return std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1])); };
  long steps = 0;
  const long max_steps = 30L * std::max(n, 1);
  int m = n - 1;
  while (m > 0) {
    if (small(m - 1)) {
      e[m - 1] = 0.0;
      --m;
      continue;
    }
    int l = m - 1;
    while (l > 0 && !small(l - 1)) --l;
    if (l > 0) e[l - 1] = 0.0;
    if (++steps > max_steps) return false;
    // shift: the eigenvalue of the trailing 2 x 2 block nearer to d[m]
    const double delta = 0.5 * (d[m - 1] - d[m]);
    const double b = e[m - 1];
    const double mu = d[m] - b * b / (delta + std::copysign(std::hypot(delta, b), delta));
    double x = d[l] - mu, z = e[l];
    for (int k = l; k < m; ++k) {
      // rotation of rows/columns k, k+1 that zeroes z against x
      const double r = std::hypot(x, z);
      const double c = r != 0.0 ? x / r : 1.0;
      const double s = r != 0.0 ? z / r : 0.0;
      if (k > l) e[k - 1] = r;
      const double a0 = d[k], b0 = e[k], c0 = d[k + 1];
      d[k] = c * c * a0 + 2.0 * c * s * b0 + s * s * c0;
      d[k + 1] = s * s * a0 - 2.0 * c * s * b0 + c * c * c0;
      e[k] = c * s * (c0 - a0) + (c * c - s * s) * b0;
      if (k + 1 < m) {  // the rotation's fill-in (bulge) is chased down
        x = e[k];
        z = s * e[k + 1];
        e[k + 1] *= c;
      }
      double* q0 = &qt[(size_t)k * n];
      double* q1 = &qt[(size_t)(k + 1) * n];
      for (int j = 0; j < n; ++j) {
        const double a = q0[j], bq = q1[j];
        q0[j] = c * a + s * bq;
        q1[j] = -s * a + c * bq;
      }
    }
  }
  return true;
}

// w descending, V[i][k] = component i of the k-th eigenvector.
int sym_eig(int n, std::vector<double> a, double* w, double* V) {
  std::vector<double> d, e, qt;
  tridiagonalise(n, a, d, e, qt);
  if (!tridiagonal_qr(n, d, e, qt)) return pfail(HB_ERR_NOCONV, "QR iteration did not converge");
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int i, int j) { return d[i] > d[j]; });
  for (int k = 0; k < n; ++k) {
    w[k] = d[order[k]];
    const double* q = &qt[(size_t)order[k] * n];
    for (int i = 0; i < n; ++i) V[(size_t)i * n + k] = q[i];
  }
  return HB_OK;
}

// ------------------------------------------------------------ device kernels

// snapshot entry (i, l), less the base snapshot if there is one
__device__ __forceinline__ double snap(const double* __restrict__ S, const double* __restrict__ B,
                                       int64_t idx) {
  return B ? S[idx] - B[idx] : S[idx];
}

// mean[l] = (1/ns) sum_i (S - B)[i][l]; one lane per column
__global__ void __launch_bounds__(BLK)
k_pod_mean(int64_t ns, int64_t L, const double* __restrict__ S, const double* __restrict__ B,
           double* __restrict__ mean) {
  const int64_t l = (int64_t)blockIdx.x * BLK + threadIdx.x;
  if (l >= L) return;
  double s = 0.0;
  for (int64_t i = 0; i < ns; ++i) s += snap(S, B, i * L + l);
  mean[l] = s / (double)ns;
}

// G[i][j] += sum over one chunk of l of c_i[l] c_j[l], c = S - B - mean, for
// the tile pair (I, J), I <= J, numbered row by row (blockIdx.x) and the
// chunk blockIdx.y of length lc; a 64 x 64 tile per workgroup, 4 x 4 entries
// per lane, 16 entries of l per LDS stage.
__global__ void __launch_bounds__(BLK)
k_pod_gram(int64_t ns, int64_t L, int ntile, int64_t lc, const double* __restrict__ S,
           const double* __restrict__ B, const double* __restrict__ mean, double* __restrict__ G) {
  int p = (int)blockIdx.x, I = 0;
  while (p >= ntile - I) {
    p -= ntile - I;
    ++I;
  }
  const int J = I + p;
  const int64_t l0 = (int64_t)blockIdx.y * lc;
  const int64_t l1 = l0 + lc < L ? l0 + lc : L;
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int t = threadIdx.x, ty = t / 16, tx = t % 16;
  double acc[4][4] = {};
  for (int64_t ls = l0; ls < l1; ls += GK) {
    for (int q = t; q < GT * GK; q += BLK) {
      const int row = q / GK, kk = q % GK;
      const int64_t l = ls + kk;
      const int64_t gi = (int64_t)I * GT + row, gj = (int64_t)J * GT + row;
      double va = 0.0, vb = 0.0;
      if (l < l1) {
        const double m = mean[l];
        if (gi < ns) va = snap(S, B, gi * L + l) - m;
        if (gj < ns) vb = snap(S, B, gj * L + l) - m;
      }
      As[kk][row] = va;
      Bs[kk][row] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[kk][ty + 16 * u];
        b[u] = Bs[kk][tx + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t gi = (int64_t)I * GT + ty + 16 * u, gj = (int64_t)J * GT + tx + 16 * v;
      if (gi < ns && gj < ns) atomicAdd(&G[gi * ns + gj], acc[u][v]);
    }
}

// basis[k][l] = sum_i Wt[i][k] c_i[l] for the modes k0 .. k0+15 (blockIdx.y)
// of one column l per lane; Wt is ns x r.
__global__ void __launch_bounds__(BLK)
k_pod_modes(int64_t ns, int64_t L, int r, const double* __restrict__ S,
            const double* __restrict__ B, const double* __restrict__ mean,
            const double* __restrict__ Wt, double* __restrict__ basis) {
  const int64_t l = (int64_t)blockIdx.x * BLK + threadIdx.x;
  if (l >= L) return;
  const int k0 = (int)blockIdx.y * BR;
  const int nk = r - k0 < BR ? r - k0 : BR;
  const double m = mean[l];
  double acc[BR] = {};
  for (int64_t i = 0; i < ns; ++i) {
    const double c = snap(S, B, i * L + l) - m;
    const double* w = Wt + i * r + k0;
#pragma unroll
    for (int k = 0; k < BR; ++k)
      if (k < nk) acc[k] = fma(w[k], c, acc[k]);
  }
#pragma unroll
  for (int k = 0; k < BR; ++k)
    if (k < nk) basis[(int64_t)(k0 + k) * L + l] = acc[k];
}

}  // namespace

extern "C" {

int hb_sym_eig(int32_t n, const double* A, double* w, double* V) {
  if (n < 1 || n > 4096 || !A || !w || !V) return pfail(HB_ERR_ARG, "bad argument");
  std::vector<double> a(A, A + (size_t)n * n);
  for (double x : a)
    if (!std::isfinite(x)) return pfail(HB_ERR_ARG, "non-finite matrix entry");
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j)
      if (a[(size_t)i * n + j] != a[(size_t)j * n + i])
        return pfail(HB_ERR_ARG, "matrix is not symmetric");
  return sym_eig(n, std::move(a), w, V);
}

int hb_pod_fit(const double* S, const double* B, int64_t ns, int64_t L, int32_t r_max,
               double floor_rel, double* mean, double* basis, double* coef, double* lam,
               int32_t* r_out, void* stream) {
  if (!S || !mean || !basis || !coef || !lam || !r_out) return pfail(HB_ERR_ARG, "NULL argument");
  if (ns < 1 || ns > 4096 || L < 1 || r_max < 1 || r_max > ns)
    return pfail(HB_ERR_ARG, "need 1 <= ns <= 4096, L >= 1, 1 <= r_max <= ns");
  if (!std::isfinite(floor_rel) || floor_rel < 0) return pfail(HB_ERR_ARG, "floor_rel must be >= 0");
  hipStream_t st = (hipStream_t)stream;
  const unsigned gl = (unsigned)((L + BLK - 1) / BLK);
  hipLaunchKernelGGL(k_pod_mean, dim3(gl), dim3(BLK), 0, st, ns, L, S, B, mean);
  HB_PCHECK(hipGetLastError());
  hb::DeviceArray<double> G;
  HB_PCHECK(G.ensure((size_t)ns * ns));
  HB_PCHECK(hipMemsetAsync(G.p, 0, G.bytes(), st));
  const int ntile = (int)((ns + GT - 1) / GT);
  const int64_t npair = (int64_t)ntile * (ntile + 1) / 2;
  int64_t chunks = (2048 + npair - 1) / npair;
  chunks = std::max<int64_t>(1, std::min<int64_t>({chunks, (L + GK - 1) / GK, 65535}));
  int64_t lc = (L + chunks - 1) / chunks;
  lc = (lc + GK - 1) / GK * GK;
  chunks = (L + lc - 1) / lc;
  hipLaunchKernelGGL(k_pod_gram, dim3((unsigned)npair, (unsigned)chunks), dim3(BLK), 0, st, ns, L,
                     ntile, lc, S, B, mean, G.p);
  HB_PCHECK(hipGetLastError());
  std::vector<double> Gh((size_t)ns * ns);
  HB_PCHECK(hipMemcpyAsync(Gh.data(), G.p, G.bytes(), hipMemcpyDeviceToHost, st));
  HB_PCHECK(hipStreamSynchronize(st));
  for (int64_t i = 0; i < ns; ++i)  // the upper triangle holds every pair
    for (int64_t j = 0; j < i; ++j) Gh[i * ns + j] = Gh[j * ns + i];
  for (double x : Gh)
    if (!std::isfinite(x)) return pfail(HB_ERR_NAN, "non-finite snapshot Gram matrix");
  std::vector<double> V((size_t)ns * ns);
  int rc = sym_eig((int)ns, std::move(Gh), lam, V.data());
  if (rc) return rc;
  int r = 0;
  while (r < r_max && lam[r] > 0.0 && lam[r] > floor_rel * lam[0]) ++r;
  for (int64_t i = 0; i < ns; ++i)
    for (int k = 0; k < r_max; ++k)
      coef[i * r_max + k] = k < r ? V[i * ns + k] * std::sqrt(lam[k]) : 0.0;
  if (r > 0) {
    std::vector<double> Wh((size_t)ns * r);
    for (int64_t i = 0; i < ns; ++i)
      for (int k = 0; k < r; ++k) Wh[i * r + k] = V[i * ns + k] / std::sqrt(lam[k]);
    hb::DeviceArray<double> W;
    HB_PCHECK(W.ensure(Wh.size()));
    HB_PCHECK(hipMemcpyAsync(W.p, Wh.data(), W.bytes(), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_pod_modes, dim3(gl, (unsigned)((r + BR - 1) / BR)), dim3(BLK), 0, st, ns,
                       L, r, S, B, mean, W.p, basis);
    HB_PCHECK(hipGetLastError());
    HB_PCHECK(hipStreamSynchronize(st));
  }
  *r_out = r;
  return HB_OK;
}

}  // extern "C"
