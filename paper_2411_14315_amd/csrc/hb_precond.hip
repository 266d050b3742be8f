// Mean-flow modal preconditioner for the Newton-GMRES solve of the HB
// equations (Section 2.3 of arXiv 2411.14315 preconditions its GMRES with the
// Jacobi diagonal of the tangent P; this is a stronger, spatially coupled
// replacement that changes iteration counts, not the root).
//
// The tangent of eq. Rmc with frozen advection and frozen tau (the paper's P
// of eq. K_mat plus the Galerkin time term C of eq. ctangent and the
// stabilisation's time terms that the paper drops) couples samples only
// through H.  Replacing every time-diagonal coefficient by its mean over
// the samples (the circulant projection of the operator in time) leaves an
// operator that the DFT block-diagonalises: Fourier mode m (H -> i m w)
// sees, per node pair (A, B),
//
//   velocity-velocity  kappa = K + sigma M + (m w)^2 rho T + i m w (rho M + Xs)   (x I3)
//   velocity-pressure  g_i   = G_i - i m w G'_i
//   pressure-velocity  d_j   = D_j + i m w D'_j
//   pressure-pressure  l     = L
//
// with sample means of  K = int rho N_A u.grad N_B + mu grad N_A.grad N_B
// + rho tau (u.grad N_A)(u.grad N_B);  G_i = -int d_i N_A N_B + tau
// (u.grad N_A) d_i N_B;  D_j = int N_A d_j N_B + tau d_j N_A (u.grad N_B);
// L = int tau/rho grad N_A.grad N_B  (eq. K_mat);  M = int N_A N_B;
// T = int tau N_A N_B;  Xs = int rho tau ((u.grad N_A) N_B - N_A (u.grad N_B));
// G'_i = int tau N_A d_i N_B;  D'_i = int tau d_i N_A N_B;  sigma = the
// pseudo-time mass coefficient.  Dirichlet velocity rows are identity and
// Dirichlet velocity columns are dropped.
//
// Each mode's complex system is approximated by V-cycles of an aggregation
// multigrid on the node graph: aggregates from two passes of pairwise
// matching (or of a node and its free neighbours), piecewise-constant
// transfer with a weighted coarse correction, Galerkin coarse operators (the 17
// coefficient fields above are summed over aggregate pairs, so every level
// has the same form), smoothing with the closed-form inverse of the 4 x 4
// nodal block, and a dense complex inverse on the
// coarsest level (damped block Jacobi, or symmetric block Gauss-Seidel over
// the colour classes of each level's graph; V- or W-cycles).  All K+1 modes
// are processed by every launch: the matrix
// coefficients are read once per node pair and applied to the K+1 mode
// vectors of the neighbour.
#include "hb.h"
#include "hb_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <memory>
#include <vector>

namespace hb {

namespace {

constexpr int PBLK = 256;
// coefficient fields per node pair (stride PC_NF doubles)
enum {
  F_K = 0, F_M = 1, F_T = 2, F_XS = 3, F_G = 4, F_D = 7, F_GP = 10, F_DP = 13, F_L = 16,
  PC_NFIELDS = 17, PC_NF = 18
};
// modes held in registers by the one-lane-per-node kernels
constexpr int PC_MM = 12;
// largest coarsest level (nodes) the dense per-mode inverse accepts
constexpr int64_t kMaxCoarse = 2048;
constexpr double QA_ = 0.58541019662496845446137605030969;
constexpr double QB_ = 0.13819660112501051517954131656344;

template <typename T>
struct cplxT {
  T re, im;
};
template <typename T>
__device__ __forceinline__ cplxT<T> cmul(cplxT<T> a, cplxT<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplxT<T> cadd(cplxT<T> a, cplxT<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ __forceinline__ cplxT<T> csub(cplxT<T> a, cplxT<T> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename T>
__device__ __forceinline__ cplxT<T> cdiv(cplxT<T> a, cplxT<T> b) {
  const T d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
using cplx = cplxT<double>;

// Position of column c in row r of a CSR graph with sorted columns.
__device__ __forceinline__ int64_t csr_find(const int32_t* __restrict__ rowptr,
                                            const int32_t* __restrict__ col, int32_t r,
                                            int32_t c) {
  int lo = rowptr[r], hi = rowptr[r + 1] - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (col[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Fine-level coefficients: one lane per tetrahedron.  Sample means of the
// quadrature-point quantities tau, tau u, tau u u^T and u are formed first
// (13 per quadrature point); every node pair's 17 fields follow from them
// and are added to the pair's CSR entry.
__global__ void __launch_bounds__(PBLK)
k_pc_assemble(int64_t ne, int64_t n, int N, const int32_t* __restrict__ tets,
              const double* __restrict__ geo, const double* __restrict__ Sy,
              const uint8_t* __restrict__ dmask, const int32_t* __restrict__ rowptr,
              const int32_t* __restrict__ col, double* __restrict__ val, Phys p) {
  const int64_t t = (int64_t)blockIdx.x * PBLK + threadIdx.x;
  if (t >= ne) return;
  int32_t a[4];
#pragma unroll
  for (int A = 0; A < 4; ++A) a[A] = tets[A * ne + t];
  double g[4][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    g[1][i] = geo[(GEO_G1 + i) * ne + t];
    g[2][i] = geo[(GEO_G2 + i) * ne + t];
    g[3][i] = geo[(GEO_G3 + i) * ne + t];
    g[0][i] = geo[(GEO_G0 + i) * ne + t];
  }
  const double V = geo[GEO_V * ne + t];
  const double x00 = geo[GEO_XI00 * ne + t], x01 = geo[GEO_XI01 * ne + t],
               x02 = geo[GEO_XI02 * ne + t], x11 = geo[GEO_XI11 * ne + t],
               x12 = geo[GEO_XI12 * ne + t], x22 = geo[GEO_XI22 * ne + t];
  const double kap0 = p.C_I * p.nu * p.nu * geo[GEO_XIXI * ne + t] + p.tau_add;
  // per quadrature point q: tau, tau u (3), tau u u^T (6: 00 01 02 11 12 22), u (3)
  double mt[4], mtu[4][3], mtuu[4][6], mu_[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    mt[q] = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) mtu[q][i] = mu_[q][i] = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) mtuu[q][i] = 0.0;
  }
  for (int s = 0; s < N; ++s) {
    double u[4][3];
#pragma unroll
    for (int A = 0; A < 4; ++A)
#pragma unroll
      for (int i = 0; i < 3; ++i) u[A][i] = Sy[((int64_t)a[A] * NCH + i) * N + s];
    double usum[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) usum[i] = u[0][i] + u[1][i] + u[2][i] + u[3][i];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double uq[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) uq[i] = QB_ * usum[i] + (QA_ - QB_) * u[q][i];
      const double kap = uq[0] * (x00 * uq[0] + x01 * uq[1] + x02 * uq[2]) +
                         uq[1] * (x01 * uq[0] + x11 * uq[1] + x12 * uq[2]) +
                         uq[2] * (x02 * uq[0] + x12 * uq[1] + x22 * uq[2]) + kap0;
      const double tau = 1.0 / sqrt(kap);
      mt[q] += tau;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        mtu[q][i] += tau * uq[i];
        mu_[q][i] += uq[i];
      }
      mtuu[q][0] += tau * uq[0] * uq[0];
      mtuu[q][1] += tau * uq[0] * uq[1];
      mtuu[q][2] += tau * uq[0] * uq[2];
      mtuu[q][3] += tau * uq[1] * uq[1];
      mtuu[q][4] += tau * uq[1] * uq[2];
      mtuu[q][5] += tau * uq[2] * uq[2];
    }
  }
  const double wq = 0.25 * V / (double)N;  // quadrature weight and sample mean
  const double rho = p.rho;
  bool dir[4];
#pragma unroll
  for (int A = 0; A < 4; ++A) dir[A] = dmask[a[A]] != 0;
  for (int A = 0; A < 4; ++A) {
    for (int B = 0; B < 4; ++B) {
      double f[PC_NFIELDS];
#pragma unroll
      for (int k = 0; k < PC_NFIELDS; ++k) f[k] = 0.0;
      const double gg = g[A][0] * g[B][0] + g[A][1] * g[B][1] + g[A][2] * g[B][2];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double NA = A == q ? QA_ : QB_;
        const double NB = B == q ? QA_ : QB_;
        const double ucB = mu_[q][0] * g[B][0] + mu_[q][1] * g[B][1] + mu_[q][2] * g[B][2];
        const double tcA = mtu[q][0] * g[A][0] + mtu[q][1] * g[A][1] + mtu[q][2] * g[A][2];
        const double tcB = mtu[q][0] * g[B][0] + mtu[q][1] * g[B][1] + mtu[q][2] * g[B][2];
        const double* T6 = mtuu[q];
        const double tuuB0 = T6[0] * g[B][0] + T6[1] * g[B][1] + T6[2] * g[B][2];
        const double tuuB1 = T6[1] * g[B][0] + T6[3] * g[B][1] + T6[4] * g[B][2];
        const double tuuB2 = T6[2] * g[B][0] + T6[4] * g[B][1] + T6[5] * g[B][2];
        const double supg = g[A][0] * tuuB0 + g[A][1] * tuuB1 + g[A][2] * tuuB2;
        f[F_K] += wq * rho * (NA * ucB + supg);
        f[F_T] += wq * mt[q] * NA * NB;
        f[F_XS] += wq * rho * (tcA * NB - NA * tcB);
        f[F_L] += wq * mt[q] * gg / rho;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          f[F_G + i] += wq * (-(double)N * g[A][i] * NB + tcA * g[B][i]);
          f[F_D + i] += wq * ((double)N * NA * g[B][i] + tcB * g[A][i]);
          f[F_GP + i] += wq * mt[q] * NA * g[B][i];
          f[F_DP + i] += wq * mt[q] * g[A][i] * NB;
        }
      }
      f[F_K] += p.mu * V * gg;
      f[F_M] = V * (A == B ? 2.0 : 1.0) / 20.0;
      if (dir[A]) {  // Dirichlet velocity row
        f[F_K] = f[F_M] = f[F_T] = f[F_XS] = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) f[F_G + i] = f[F_GP + i] = 0.0;
      }
      if (dir[B]) {  // Dirichlet velocity column
        f[F_K] = f[F_M] = f[F_T] = f[F_XS] = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) f[F_D + i] = f[F_DP + i] = 0.0;
      }
      double* v = val + csr_find(rowptr, col, a[A], a[B]) * PC_NF;
#pragma unroll
      for (int k = 0; k < PC_NFIELDS; ++k)
        if (f[k] != 0.0) unsafeAtomicAdd(v + k, f[k]);
    }
  }
}

// Identity velocity block on the diagonal of Dirichlet rows.
__global__ void __launch_bounds__(PBLK)
k_pc_dirichlet(int64_t n, const uint8_t* __restrict__ dmask, const int32_t* __restrict__ diag,
               double* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * PBLK + threadIdx.x;
  if (i >= n || !dmask[i]) return;
  val[(int64_t)diag[i] * PC_NF + F_K] = 1.0;
}

// Galerkin coarse coefficients: each coarse entry sums the fine entries of
// its aggregate pair (a gather over a precomputed list: no atomics).
__global__ void __launch_bounds__(PBLK)
k_pc_galerkin(int64_t nnz_c, const int32_t* __restrict__ gptr, const int32_t* __restrict__ gsrc,
              const double* __restrict__ vf, double* __restrict__ vc) {
  const int64_t gid = (int64_t)blockIdx.x * PBLK + threadIdx.x;
  if (gid >= nnz_c * PC_NFIELDS) return;
  const int64_t k = gid / PC_NFIELDS;
  const int f = (int)(gid - k * PC_NFIELDS);
  double s = 0.0;
  for (int j = gptr[k]; j < gptr[k + 1]; ++j) s += vf[(int64_t)gsrc[j] * PC_NF + f];
  vc[k * PC_NF + f] = s;
}

struct Coef {
  double sigma, rho, omega;
  int nm;
};

// The mode-m coefficients of one node pair (T: arithmetic type, M: the type
// the coefficients are stored in).
template <typename T>
struct PairOp {
  cplxT<T> kap, g[3], d[3];
  T l;
};
template <typename T, typename M>
__device__ __forceinline__ PairOp<T> pair_op(const M* __restrict__ v, const Coef& c, T s) {
  PairOp<T> o;
  const T rho = (T)c.rho;
  o.kap = {(T)v[F_K] + (T)c.sigma * (T)v[F_M] + s * s * rho * (T)v[F_T],
           s * (rho * (T)v[F_M] + (T)v[F_XS])};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    o.g[i] = {(T)v[F_G + i], -s * (T)v[F_GP + i]};
    o.d[i] = {(T)v[F_D + i], s * (T)v[F_DP + i]};
  }
  o.l = (T)v[F_L];
  return o;
}

// Complex vectors: [node][mode][4][re, im].
template <typename T>
__device__ __forceinline__ void load4(const T* __restrict__ x, int64_t idx, cplxT<T> out[4]) {
  const T* p = x + idx * 8;
#pragma unroll
  for (int f = 0; f < 4; ++f) out[f] = {p[2 * f], p[2 * f + 1]};
}
template <typename T>
__device__ __forceinline__ void store4(T* __restrict__ x, int64_t idx, const cplxT<T> v[4]) {
  T* p = x + idx * 8;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    p[2 * f] = v[f].re;
    p[2 * f + 1] = v[f].im;
  }
}

// e = D^-1 r for the nodal block D = [kap I, g; d^T, l] (Schur complement on
// the pressure).
template <typename T>
__device__ __forceinline__ void block_solve(const PairOp<T>& o, const cplxT<T> r[4],
                                            cplxT<T> e[4]) {
  cplxT<T> sp = r[3], den = {o.l, (T)0};
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    sp = csub(sp, cdiv(cmul(o.d[f], r[f]), o.kap));
    den = csub(den, cdiv(cmul(o.d[f], o.g[f]), o.kap));
  }
  e[3] = cdiv(sp, den);
#pragma unroll
  for (int f = 0; f < 3; ++f) e[f] = cdiv(csub(r[f], cmul(o.g[f], e[3])), o.kap);
}

// A pending coarse-level correction of x: the fine vector is read as
// x_j + gamma xc[agg[j]] (xc = NULL: plain x).
template <typename T>
struct Corr {
  const T* xc;
  const int32_t* agg;
  T gamma;
};
template <typename T>
__device__ __forceinline__ void load_x(const T* __restrict__ x, const Corr<T>& cr, int64_t j,
                                       int m, int nm, cplxT<T> out[4]) {
  load4(x, j * nm + m, out);
  if (cr.xc) {
    cplxT<T> e[4];
    load4(cr.xc, (int64_t)cr.agg[j] * nm + m, e);
#pragma unroll
    for (int f = 0; f < 4; ++f) out[f] = {out[f].re + cr.gamma * e[f].re, out[f].im + cr.gamma * e[f].im};
  }
}

// acc += A_row(i) x for one mode
template <typename T, typename M>
__device__ __forceinline__ void row_apply(int64_t i, int m, const int32_t* __restrict__ rowptr,
                                          const int32_t* __restrict__ col,
                                          const M* __restrict__ val, const Coef& c, T s,
                                          const T* __restrict__ x, const Corr<T>& cr,
                                          cplxT<T> acc[4]) {
  for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
    const int64_t j = col[k];
    const PairOp<T> o = pair_op<T, M>(val + (int64_t)k * PC_NF, c, s);
    cplxT<T> xj[4];
    load_x(x, cr, j, m, c.nm, xj);
#pragma unroll
    for (int f = 0; f < 3; ++f)
      acc[f] = cadd(acc[f], cadd(cmul(o.kap, xj[f]), cmul(o.g[f], xj[3])));
    acc[3] = cadd(acc[3], cadd(cadd(cmul(o.d[0], xj[0]), cmul(o.d[1], xj[1])),
                               cadd(cmul(o.d[2], xj[2]), cplxT<T>{o.l * xj[3].re, o.l * xj[3].im})));
  }
}

// Row operation on all modes, one lane per (node, mode):
//   OP 0: y = A x;  OP 1: y = b - A x;
//   OP 2: y = x + w D^-1 (b - A x) (x = NULL: y = w D^-1 b), D the nodal block;
// with a pending coarse correction cr, x stands for x + gamma P xc.
template <int OP, typename T, typename M>
__global__ void __launch_bounds__(PBLK)
k_pc_rows(int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
          const int32_t* __restrict__ diag, const M* __restrict__ val, Coef c,
          const T* __restrict__ b, const T* __restrict__ x, T* __restrict__ y, double wj,
          Corr<T> cr) {
  const int64_t gid = (int64_t)blockIdx.x * PBLK + threadIdx.x;
  if (gid >= n * c.nm) return;
  const int64_t i = gid / c.nm;
  const int m = (int)(gid - i * c.nm);
  const T s = (T)(m * c.omega);
  cplxT<T> acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  if (x) row_apply<T, M>(i, m, rowptr, col, val, c, s, x, cr, acc);
  if (OP == 0) {
    store4(y, gid, acc);
    return;
  }
  cplxT<T> r[4];
  load4(b, gid, r);
#pragma unroll
  for (int f = 0; f < 4; ++f) r[f] = csub(r[f], acc[f]);
  if (OP == 1) {
    store4(y, gid, r);
    return;
  }
  cplxT<T> e[4];
  block_solve(pair_op<T, M>(val + (int64_t)diag[i] * PC_NF, c, s), r, e);
  cplxT<T> out[4];
  if (x) load_x(x, cr, i, m, c.nm, out);
  else out[0] = out[1] = out[2] = out[3] = {(T)0, (T)0};
  const T w = (T)wj;
#pragma unroll
  for (int f = 0; f < 4; ++f) out[f] = {out[f].re + w * e[f].re, out[f].im + w * e[f].im};
  store4(y, gid, out);
}

// Gauss-Seidel sweep over one colour class (no two rows of a class are
// neighbours, so the class updates x in place without races): for each row
// i of the class and each mode, x_i += D_i^-1 (b - A x)_i.
template <typename T, typename M>
__global__ void __launch_bounds__(PBLK)
k_pc_gs(int64_t nrows, const int32_t* __restrict__ rows, const int32_t* __restrict__ rowptr,
        const int32_t* __restrict__ col, const int32_t* __restrict__ diag,
        const M* __restrict__ val, Coef c, const T* __restrict__ b, T* x) {
  const int64_t gid = (int64_t)blockIdx.x * PBLK + threadIdx.x;
  if (gid >= nrows * c.nm) return;
  const int64_t li = gid / c.nm;
  const int m = (int)(gid - li * c.nm);
  const int64_t i = rows[li];
  const T s = (T)(m * c.omega);
  cplxT<T> acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  row_apply<T, M>(i, m, rowptr, col, val, c, s, x, Corr<T>{nullptr, nullptr, (T)0}, acc);
  cplxT<T> r[4];
  load4(b, i * c.nm + m, r);
#pragma unroll
  for (int f = 0; f < 4; ++f) r[f] = csub(r[f], acc[f]);
  cplxT<T> e[4];
  block_solve(pair_op<T, M>(val + (int64_t)diag[i] * PC_NF, c, s), r, e);
  cplxT<T> xi[4];
  load4(x, i * c.nm + m, xi);
#pragma unroll
  for (int f = 0; f < 4; ++f) xi[f] = cadd(xi[f], e[f]);
  store4(x, i * c.nm + m, xi);
}

template <typename T>
__global__ void __launch_bounds__(PBLK) k_pc_zero(int64_t len, T* __restrict__ x) {
  const int64_t gid = (int64_t)blockIdx.x * PBLK + threadIdx.x;
  if (gid < len) x[gid] = (T)0;
}

// FP32 copy of the coefficients for the smoothing and transfer kernels.
__global__ void __launch_bounds__(PBLK)
k_pc_narrow(int64_t len, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t gid = (int64_t)blockIdx.x * PBLK + threadIdx.x;
  if (gid < len) b[gid] = (float)a[gid];
}

// bc[I] = sum of r over the members of aggregate I (all modes).
template <typename T>
__global__ void __launch_bounds__(PBLK)
k_pc_restrict(int64_t nc, int nm, const int32_t* __restrict__ mptr,
              const int32_t* __restrict__ mem, const T* __restrict__ r, T* __restrict__ bc) {
  const int64_t gid = (int64_t)blockIdx.x * PBLK + threadIdx.x;
  if (gid >= nc * nm * 8) return;
  const int64_t I = gid / (nm * 8);
  const int k = (int)(gid - I * nm * 8);
  T s = (T)0;
  for (int j = mptr[I]; j < mptr[I + 1]; ++j) s += r[(int64_t)mem[j] * nm * 8 + k];
  bc[gid] = s;
}

// x[i] += gamma xc[agg[i]] (all modes).
template <typename T>
__global__ void __launch_bounds__(PBLK)
k_pc_prolong(int64_t n, int nm, const int32_t* __restrict__ agg, const T* __restrict__ xc,
             T* __restrict__ x, double gamma) {
  const int64_t gid = (int64_t)blockIdx.x * PBLK + threadIdx.x;
  if (gid >= n * nm * 8) return;
  const int64_t i = gid / (nm * 8);
  const int k = (int)(gid - i * nm * 8);
  x[gid] += (T)gamma * xc[(int64_t)agg[i] * nm * 8 + k];
}

// Dense coarsest-level matrices, one per mode: A[m][4I+a][4J+b] (complex,
// row-major, D = 4 nc), filled from the CSR coefficients.  A must be zero.
__global__ void __launch_bounds__(PBLK)
k_pc_dense(int64_t nc, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
           const double* __restrict__ val, Coef c, double* __restrict__ A) {
  const int64_t nnz = rowptr[nc];
  const int64_t gid = (int64_t)blockIdx.x * PBLK + threadIdx.x;
  if (gid >= nnz * c.nm) return;
  const int64_t k = gid / c.nm;
  const int m = (int)(gid - k * c.nm);
  // row of entry k
  int lo = 0, hi = (int)nc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rowptr[mid] <= k) lo = mid;
    else hi = mid - 1;
  }
  const int64_t I = lo, J = col[k];
  const int64_t D = 4 * nc;
  const PairOp<double> o = pair_op<double, double>(val + k * PC_NF, c, m * c.omega);
  double* Am = A + (int64_t)m * D * D * 2;
  auto put = [&](int64_t r, int64_t cc, cplx v) {
    Am[(r * D + cc) * 2] = v.re;
    Am[(r * D + cc) * 2 + 1] = v.im;
  };
  for (int f = 0; f < 3; ++f) {
    put(4 * I + f, 4 * J + f, o.kap);
    put(4 * I + f, 4 * J + 3, o.g[f]);
    put(4 * I + 3, 4 * J + f, o.d[f]);
  }
  put(4 * I + 3, 4 * J + 3, {o.l, 0.0});
}

// In-place Gauss-Jordan inversion with partial pivoting of one D x D
// complex matrix per workgroup (mode = blockIdx.x); W holds [D][2D]
// (matrix | identity) and receives [I | A^-1]; the inverse is copied to Ainv.
__global__ void __launch_bounds__(PBLK)
k_pc_invert(int D, const double* __restrict__ A, double* __restrict__ W,
            double* __restrict__ Ainv, int* __restrict__ singular) {
  const int m = blockIdx.x;
  const double* Am = A + (int64_t)m * D * D * 2;
  double* Wm = W + (int64_t)m * D * 2 * D * 2;
  const int W2 = 2 * D;
  for (int64_t e = threadIdx.x; e < (int64_t)D * W2; e += PBLK) {
    const int r = (int)(e / W2), cc = (int)(e - (int64_t)r * W2);
    double re = 0.0, im = 0.0;
    if (cc < D) {
      re = Am[((int64_t)r * D + cc) * 2];
      im = Am[((int64_t)r * D + cc) * 2 + 1];
    } else if (cc - D == r) {
      re = 1.0;
    }
    Wm[e * 2] = re;
    Wm[e * 2 + 1] = im;
  }
  __shared__ double smax[PBLK];
  __shared__ int sidx[PBLK];
  __shared__ double piv[2];
  __syncthreads();
  for (int k = 0; k < D; ++k) {
    // pivot search in column k, rows k..D-1
    double best = -1.0;
    int bi = k;
    for (int r = k + threadIdx.x; r < D; r += PBLK) {
      const double* w = Wm + ((int64_t)r * W2 + k) * 2;
      const double a = w[0] * w[0] + w[1] * w[1];
      if (a > best) {
        best = a;
        bi = r;
      }
    }
    smax[threadIdx.x] = best;
    sidx[threadIdx.x] = bi;
    __syncthreads();
    for (int off = PBLK / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off && smax[threadIdx.x + off] > smax[threadIdx.x]) {
        smax[threadIdx.x] = smax[threadIdx.x + off];
        sidx[threadIdx.x] = sidx[threadIdx.x + off];
      }
      __syncthreads();
    }
    const int pr = sidx[0];
    if (!(smax[0] > 0.0)) {
      if (threadIdx.x == 0) atomicOr(singular, 1);
      return;  // uniform across the workgroup
    }
    // swap rows k and pr
    if (pr != k)
      for (int cc = threadIdx.x; cc < W2; cc += PBLK) {
        double* a = Wm + ((int64_t)k * W2 + cc) * 2;
        double* b2 = Wm + ((int64_t)pr * W2 + cc) * 2;
        const double t0 = a[0], t1 = a[1];
        a[0] = b2[0];
        a[1] = b2[1];
        b2[0] = t0;
        b2[1] = t1;
      }
    __syncthreads();
    if (threadIdx.x == 0) {
      const double* w = Wm + ((int64_t)k * W2 + k) * 2;
      const double d = w[0] * w[0] + w[1] * w[1];
      piv[0] = w[0] / d;
      piv[1] = -w[1] / d;
    }
    __syncthreads();
    const cplx ip = {piv[0], piv[1]};
    for (int cc = threadIdx.x; cc < W2; cc += PBLK) {
      double* a = Wm + ((int64_t)k * W2 + cc) * 2;
      const cplx v = cmul(cplx{a[0], a[1]}, ip);
      a[0] = v.re;
      a[1] = v.im;
    }
    __syncthreads();
    // eliminate column k from every other row
    for (int64_t e = threadIdx.x; e < (int64_t)D * W2; e += PBLK) {
      const int r = (int)(e / W2), cc = (int)(e - (int64_t)r * W2);
      if (r == k || cc == k) continue;
      const double* fr = Wm + ((int64_t)r * W2 + k) * 2;
      const double* pk = Wm + ((int64_t)k * W2 + cc) * 2;
      double* a = Wm + e * 2;
      const cplx v = csub(cplx{a[0], a[1]}, cmul(cplx{fr[0], fr[1]}, cplx{pk[0], pk[1]}));
      a[0] = v.re;
      a[1] = v.im;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < D; r += PBLK)
      if (r != k) {
        double* a = Wm + ((int64_t)r * W2 + k) * 2;
        a[0] = 0.0;
        a[1] = 0.0;
      }
    __syncthreads();
  }
  double* Im = Ainv + (int64_t)m * D * D * 2;
  for (int64_t e = threadIdx.x; e < (int64_t)D * D; e += PBLK) {
    const int r = (int)(e / D), cc = (int)(e - (int64_t)r * D);
    Im[e * 2] = Wm[((int64_t)r * W2 + D + cc) * 2];
    Im[e * 2 + 1] = Wm[((int64_t)r * W2 + D + cc) * 2 + 1];
  }
}

// x = Ainv_m b on the coarsest level (FP64 arithmetic); one lane per (mode, row).
template <typename T>
__global__ void __launch_bounds__(PBLK)
k_pc_dense_apply(int64_t nc, int nm, const double* __restrict__ Ainv, const T* __restrict__ b,
                 T* __restrict__ x) {
  const int64_t D = 4 * nc;
  const int64_t gid = (int64_t)blockIdx.x * PBLK + threadIdx.x;
  if (gid >= D * nm) return;
  const int m = (int)(gid / D);
  const int64_t r = gid - (int64_t)m * D;
  const double* Ar = Ainv + ((int64_t)m * D * D + r * D) * 2;
  double re = 0.0, im = 0.0;
  for (int64_t cc = 0; cc < D; ++cc) {
    const int64_t J = cc >> 2;
    const int f = (int)(cc & 3);
    const T* bv = b + ((J * nm + m) * 4 + f) * 2;
    const double br = (double)bv[0], bi = (double)bv[1];
    re += Ar[cc * 2] * br - Ar[cc * 2 + 1] * bi;
    im += Ar[cc * 2] * bi + Ar[cc * 2 + 1] * br;
  }
  const int64_t I = r >> 2;
  const int f = (int)(r & 3);
  T* xv = x + ((I * nm + m) * 4 + f) * 2;
  xv[0] = (T)re;
  xv[1] = (T)im;
}

// Samples -> modes: b[a][m][f] = (1/N) sum_s q[a][f][s] e^{-2 pi i m s / N}
// (m = 0..K); q has in_ch channels per node.  A workgroup takes PC_TN
// nodes: their 4 N samples are staged in LDS with contiguous loads, one lane
// per (node, field) transforms with all modes in registers (K + 1 <= PC_MM;
// the table index is uniform across the wavefront), and the modal tile goes
// back through LDS to contiguous stores.  LDS: PC_TN max(4 N, 8 (K + 1))
// values.
constexpr int PC_TN = PBLK / 4;
template <typename TQ, typename T>
__global__ void __launch_bounds__(PBLK)
k_pc_to_modes(int64_t n, int N, int nm, const TQ* __restrict__ q, int in_ch,
              const double* __restrict__ cs, T* __restrict__ b) {
  extern __shared__ double sbuf[];
  const int64_t a0 = (int64_t)blockIdx.x * PC_TN;
  const int tn = (int)min<int64_t>(PC_TN, n - a0);
  const int t = threadIdx.x;
  const int NS = 4 * N;
  for (int idx = t; idx < tn * NS; idx += PBLK) {
    const int al = idx / NS;
    sbuf[idx] = (double)q[(a0 + al) * in_ch * N + (idx - al * NS)];
  }
  __syncthreads();
  const int al = t >> 2, f = t & 3;
  double re[PC_MM], im[PC_MM];
#pragma unroll
  for (int m = 0; m < PC_MM; ++m) re[m] = im[m] = 0.0;
  if (al < tn) {
    const double* qa = sbuf + (al * 4 + f) * N;
    for (int s = 0; s < N; ++s) {
      const double v = qa[s];
#pragma unroll
      for (int m = 0; m < PC_MM; ++m)
        if (m < nm) {
          re[m] += v * cs[(m * N + s) * 2];
          im[m] -= v * cs[(m * N + s) * 2 + 1];
        }
    }
  }
  __syncthreads();
  const double inv = 1.0 / N;
  if (al < tn) {
#pragma unroll
    for (int m = 0; m < PC_MM; ++m)
      if (m < nm) {
        double* p = sbuf + ((al * nm + m) * 4 + f) * 2;
        p[0] = re[m] * inv;
        p[1] = im[m] * inv;
      }
  }
  __syncthreads();
  T* bt = b + a0 * nm * 8;
  for (int idx = t; idx < tn * nm * 8; idx += PBLK) bt[idx] = (T)sbuf[idx];
}

// The same for any K: one lane per (node, mode).
template <typename TQ, typename T>
__global__ void __launch_bounds__(PBLK)
k_pc_to_modes_wide(int64_t n, int N, int nm, const TQ* __restrict__ q, int in_ch,
                   const double* __restrict__ cs, T* __restrict__ b) {
  const int64_t gid = (int64_t)blockIdx.x * PBLK + threadIdx.x;
  if (gid >= n * nm) return;
  const int64_t a = gid / nm;
  const int m = (int)(gid - a * nm);
  cplxT<T> out[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    double re = 0.0, im = 0.0;
    const TQ* qa = q + (a * in_ch + f) * N;
    for (int s = 0; s < N; ++s) {
      const double v = (double)qa[s];
      re += v * cs[(m * N + s) * 2];
      im -= v * cs[(m * N + s) * 2 + 1];
    }
    out[f] = {(T)(re / N), (T)(im / N)};
  }
  store4(b, gid, out);
}

// Modes -> samples: z[a][f][s] = Re x_0 + 2 sum_{m>=1} Re(x_m e^{2 pi i m s/N}).
// Staged like k_pc_to_modes: the tile's modes in through LDS, one lane per
// (node, field) with the modes in registers (K + 1 <= PC_MM), the samples
// out through LDS.
template <typename T, typename TZ>
__global__ void __launch_bounds__(PBLK)
k_pc_from_modes(int64_t n, int N, int nm, const T* __restrict__ x,
                const double* __restrict__ cs, TZ* __restrict__ z) {
  extern __shared__ double sbuf[];
  const int64_t a0 = (int64_t)blockIdx.x * PC_TN;
  const int tn = (int)min<int64_t>(PC_TN, n - a0);
  const int t = threadIdx.x;
  const T* xt = x + a0 * nm * 8;
  for (int idx = t; idx < tn * nm * 8; idx += PBLK) sbuf[idx] = (double)xt[idx];
  __syncthreads();
  const int al = t >> 2, f = t & 3;
  double xr[PC_MM], xi[PC_MM];
#pragma unroll
  for (int m = 0; m < PC_MM; ++m) {
    xr[m] = xi[m] = 0.0;
    if (al < tn && m < nm) {
      const double* p = sbuf + ((al * nm + m) * 4 + f) * 2;
      xr[m] = p[0];
      xi[m] = p[1];
    }
  }
  __syncthreads();
  if (al < tn) {
    double* za = sbuf + (al * 4 + f) * N;
    for (int s = 0; s < N; ++s) {
      double v = 0.0;
#pragma unroll
      for (int m = 1; m < PC_MM; ++m)
        if (m < nm) v += xr[m] * cs[(m * N + s) * 2] - xi[m] * cs[(m * N + s) * 2 + 1];
      za[s] = xr[0] + 2.0 * v;
    }
  }
  __syncthreads();
  TZ* zt = z + a0 * 4 * N;
  for (int idx = t; idx < tn * 4 * N; idx += PBLK) zt[idx] = (TZ)sbuf[idx];
}

// The same for any K: one lane per (node, field, sample).
template <typename T, typename TZ>
__global__ void __launch_bounds__(PBLK)
k_pc_from_modes_wide(int64_t n, int N, int nm, const T* __restrict__ x,
                     const double* __restrict__ cs, TZ* __restrict__ z) {
  const int64_t gid = (int64_t)blockIdx.x * PBLK + threadIdx.x;
  if (gid >= n * 4 * N) return;
  const int64_t a = gid / (4 * N);
  const int r = (int)(gid - a * 4 * N);
  const int f = r / N;
  const int s = r - f * N;
  double v = (double)x[((a * nm + 0) * 4 + f) * 2];
  for (int m = 1; m < nm; ++m) {
    const T* xm = x + ((a * nm + m) * 4 + f) * 2;
    v += 2.0 * ((double)xm[0] * cs[(m * N + s) * 2] - (double)xm[1] * cs[(m * N + s) * 2 + 1]);
  }
  z[gid] = (TZ)v;
}

inline unsigned nblk(int64_t work) { return (unsigned)((work + PBLK - 1) / PBLK); }

// LDS of one mode-transform tile: PC_TN nodes x max(4 N, 8 (K + 1)) values
inline size_t tile_lds(int N, int nm) {
  return sizeof(double) * PC_TN * (size_t)(4 * N > 8 * nm ? 4 * N : 8 * nm);
}

template <typename TQ, typename T>
void launch_to_modes(int64_t n, int N, int nm, const TQ* q, int in_ch, const double* cs, T* b,
                     hipStream_t st) {
  if (nm <= PC_MM)
    hipLaunchKernelGGL((k_pc_to_modes<TQ, T>), dim3((unsigned)((n + PC_TN - 1) / PC_TN)),
                       dim3(PBLK), tile_lds(N, nm), st, n, N, nm, q, in_ch, cs, b);
  else
    hipLaunchKernelGGL((k_pc_to_modes_wide<TQ, T>), dim3(nblk(n * nm)), dim3(PBLK), 0, st, n, N,
                       nm, q, in_ch, cs, b);
}

template <typename T, typename TZ>
void launch_from_modes(int64_t n, int N, int nm, const T* x, const double* cs, TZ* z,
                       hipStream_t st) {
  if (nm <= PC_MM)
    hipLaunchKernelGGL((k_pc_from_modes<T, TZ>), dim3((unsigned)((n + PC_TN - 1) / PC_TN)),
                       dim3(PBLK), tile_lds(N, nm), st, n, N, nm, x, cs, z);
  else
    hipLaunchKernelGGL((k_pc_from_modes_wide<T, TZ>), dim3(nblk(n * 4 * N)), dim3(PBLK), 0, st, n,
                       N, nm, x, cs, z);
}

}  // namespace

// ---------------------------------------------------------------- hierarchy

struct PcLevel {
  int64_t n = 0, nnz = 0;
  DeviceArray<int32_t> rowptr, col, diag;
  DeviceArray<double> val;
  // transfer to the next level: aggregate of each node, members of each
  // coarse node, and the fine entries of each coarse entry
  DeviceArray<int32_t> agg, mptr, mem, gptr, gsrc;
  DeviceArray<double> x, x2, b, r;
  // FP32 copies of the coefficients and vectors for FP32 cycles
  DeviceArray<float> valf, xf, x2f, bf, rf;
  // colour classes of the level's graph (Gauss-Seidel smoothing)
  DeviceArray<int32_t> crows;
  std::vector<int64_t> cptr;
};

struct Precond {
  std::vector<PcLevel> lv;
  int nm = 0;       // modes (K + 1) the vectors are sized for
  int N = 0;
  DeviceArray<double> cs;            // [nm][N] (cos, sin) of 2 pi m s / N
  DeviceArray<double> dense, work, inv;  // coarsest level
  DeviceArray<int> flag;
  int64_t dense_D = 0;
  int nu = 2;
  int cycles = 1;
  double wj = 0.7;
  double gamma = 1.0;  // weight of the coarse-level correction
  int smoother = 0;    // 0 damped block Jacobi, 1 symmetric block Gauss-Seidel
  int wcycle = 0;      // 1: two coarse-level cycles per level (W-cycle)
  int fp32 = 0;        // 1: cycles on FP32 vectors and coefficients
  Coef coef{};
  size_t bytes() const {
    size_t b = cs.bytes() + dense.bytes() + work.bytes() + inv.bytes();
    for (const auto& l : lv)
      b += l.rowptr.bytes() + l.col.bytes() + l.diag.bytes() + l.val.bytes() + l.agg.bytes() +
           l.mptr.bytes() + l.mem.bytes() + l.gptr.bytes() + l.gsrc.bytes() + l.x.bytes() +
           l.x2.bytes() + l.b.bytes() + l.r.bytes() + l.valf.bytes() + l.xf.bytes() +
           l.x2f.bytes() + l.bf.bytes() + l.rf.bytes();
    return b;
  }
};

void precond_destroy(Precond* p) { delete p; }
size_t precond_bytes(const Precond* p) { return p ? p->bytes() : 0; }
int precond_levels(const Precond* p, int64_t* sizes, int max) {
  if (!p) return 0;
  const int L = (int)std::min<size_t>(p->lv.size(), (size_t)max);
  for (int i = 0; i < L; ++i) sizes[i] = p->lv[i].n;
  return (int)p->lv.size();
}

namespace {

struct HostGraph {
  std::vector<int32_t> rowptr, col;
};

// Node graph (with self loops, sorted columns) of a tetrahedral mesh.
HostGraph node_graph(int64_t n, int64_t ne, const std::vector<int32_t>& tets_soa) {
  std::vector<int32_t> tptr(n + 1, 0), tl(4 * ne);
  for (int64_t k = 0; k < 4 * ne; ++k) ++tptr[tets_soa[k] + 1];
  for (int64_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
  {
    std::vector<int32_t> fill(tptr.begin(), tptr.end() - 1);
    for (int64_t A = 0; A < 4; ++A)
      for (int64_t t = 0; t < ne; ++t) tl[fill[tets_soa[A * ne + t]]++] = (int32_t)t;
  }
  HostGraph g;
  g.rowptr.assign(n + 1, 0);
  g.col.reserve(16 * n);
  std::vector<int32_t> nb;
  for (int64_t i = 0; i < n; ++i) {
    nb.clear();
    nb.push_back((int32_t)i);
    for (int k = tptr[i]; k < tptr[i + 1]; ++k)
      for (int A = 0; A < 4; ++A) nb.push_back(tets_soa[A * ne + tl[k]]);
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    g.col.insert(g.col.end(), nb.begin(), nb.end());
    g.rowptr[i + 1] = (int32_t)g.col.size();
  }
  return g;
}

// Greedy aggregation: a node whose neighbours are all free starts an
// aggregate with them; the remaining nodes join a neighbouring aggregate,
// or form one of their own.
int64_t aggregate(const HostGraph& g, std::vector<int32_t>& agg) {
  const int64_t n = (int64_t)g.rowptr.size() - 1;
  agg.assign(n, -1);
  int64_t na = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    bool free = true;
    for (int k = g.rowptr[i]; k < g.rowptr[i + 1] && free; ++k) free = agg[g.col[k]] < 0;
    if (!free) continue;
    for (int k = g.rowptr[i]; k < g.rowptr[i + 1]; ++k) agg[g.col[k]] = (int32_t)na;
    ++na;
  }
  std::vector<int32_t> pass2(agg);
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    for (int k = g.rowptr[i]; k < g.rowptr[i + 1]; ++k)
      if (agg[g.col[k]] >= 0) {
        pass2[i] = agg[g.col[k]];
        break;
      }
  }
  agg.swap(pass2);
  for (int64_t i = 0; i < n; ++i)
    if (agg[i] < 0) agg[i] = (int32_t)na++;
  return na;
}

// Members of each aggregate (CSR) and the aggregated graph.
void coarsen_graph(const HostGraph& g, const std::vector<int32_t>& agg, int64_t na,
                   std::vector<int32_t>& mptr, std::vector<int32_t>& mem, HostGraph& gc) {
  const int64_t nl = (int64_t)g.rowptr.size() - 1;
  mptr.assign(na + 1, 0);
  mem.resize(nl);
  for (int64_t i = 0; i < nl; ++i) ++mptr[agg[i] + 1];
  for (int64_t I = 0; I < na; ++I) mptr[I + 1] += mptr[I];
  {
    std::vector<int32_t> fill(mptr.begin(), mptr.end() - 1);
    for (int64_t i = 0; i < nl; ++i) mem[fill[agg[i]]++] = (int32_t)i;
  }
  gc.rowptr.assign(na + 1, 0);
  gc.col.clear();
  std::vector<int32_t> nb;
  for (int64_t I = 0; I < na; ++I) {
    nb.clear();
    for (int j = mptr[I]; j < mptr[I + 1]; ++j) {
      const int32_t i = mem[j];
      for (int k = g.rowptr[i]; k < g.rowptr[i + 1]; ++k) nb.push_back(agg[g.col[k]]);
    }
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    gc.col.insert(gc.col.end(), nb.begin(), nb.end());
    gc.rowptr[I + 1] = (int32_t)gc.col.size();
  }
}

// Greedy colouring of a graph (self loops ignored): classes of rows that
// share no edge, as a permutation grouped by colour.
void colour_classes(const HostGraph& g, std::vector<int64_t>& cptr, std::vector<int32_t>& rows) {
  const int64_t n = (int64_t)g.rowptr.size() - 1;
  std::vector<int32_t> colour(n, -1);
  std::vector<int64_t> mark;
  int ncol = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int k = g.rowptr[i]; k < g.rowptr[i + 1]; ++k) {
      const int32_t c = colour[g.col[k]];
      if (c >= 0) {
        if ((int)mark.size() <= c) mark.resize(c + 1, -1);
        mark[c] = i;
      }
    }
    int c = 0;
    while (c < (int)mark.size() && mark[c] == i) ++c;
    colour[i] = c;
    ncol = std::max(ncol, c + 1);
  }
  cptr.assign(ncol + 1, 0);
  for (int64_t i = 0; i < n; ++i) ++cptr[colour[i] + 1];
  for (int c = 0; c < ncol; ++c) cptr[c + 1] += cptr[c];
  rows.resize(n);
  std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
  for (int64_t i = 0; i < n; ++i) rows[fill[colour[i]]++] = (int32_t)i;
}

// One pass of pairwise matching: each node in turn is paired with its first
// unmatched neighbour (or left alone); pairs are numbered in order.
int64_t match_pairs(const HostGraph& g, std::vector<int32_t>& agg) {
  const int64_t n = (int64_t)g.rowptr.size() - 1;
  std::vector<int32_t> mate(n, -1);
  for (int64_t i = 0; i < n; ++i) {
    if (mate[i] >= 0) continue;
    mate[i] = (int32_t)i;
    for (int k = g.rowptr[i]; k < g.rowptr[i + 1]; ++k) {
      const int32_t j = g.col[k];
      if (j != i && mate[j] < 0) {
        mate[i] = j;
        mate[j] = (int32_t)i;
        break;
      }
    }
  }
  agg.assign(n, -1);
  int64_t na = 0;
  for (int64_t i = 0; i < n; ++i)
    if (agg[i] < 0) {
      agg[i] = (int32_t)na;
      agg[mate[i]] = (int32_t)na;
      ++na;
    }
  return na;
}

// Two passes of pairwise matching: aggregates of up to four nodes.
int64_t aggregate_pairs(const HostGraph& g, std::vector<int32_t>& agg) {
  std::vector<int32_t> a1, a2, mptr, mem;
  const int64_t n1 = match_pairs(g, a1);
  HostGraph g1;
  coarsen_graph(g, a1, n1, mptr, mem, g1);
  const int64_t n2 = match_pairs(g1, a2);
  agg.resize(a1.size());
  for (size_t i = 0; i < a1.size(); ++i) agg[i] = a2[a1[i]];
  return n2;
}

template <typename T>
hipError_t upload(DeviceArray<T>& d, const std::vector<T>& h) {
  hipError_t e = d.ensure(h.size());
  if (e != hipSuccess) return e;
  if (!h.empty()) e = hipMemcpy(d.p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice);
  return e;
}

}  // namespace

namespace {

// One level of the hierarchy on the host: its node graph (CSR with self
// loops, position of the diagonal), colour classes, and the transfer to the
// next level (aggregate of each node, members of each aggregate, fine
// entries of each coarse entry); the transfer is empty on the coarsest level.
struct HostLevel {
  int64_t n = 0, nnz = 0;
  std::vector<int32_t> rowptr, col, diag, crows, agg, mptr, mem, gptr, gsrc;
  std::vector<int64_t> cptr;
};

// The hierarchy of a mesh's node graph (tets SoA [4][ne], indices < n):
// aggregation until at most coarse_max nodes remain or it stops coarsening.
void build_levels(int64_t n, int64_t ne, const std::vector<int32_t>& tets_soa, int coarse_max,
                  int pairwise, std::vector<HostLevel>& out) {
  out.clear();
  HostGraph g = node_graph(n, ne, tets_soa);
  for (int level = 0;; ++level) {
    out.emplace_back();
    HostLevel& L = out.back();
    const int64_t nl = (int64_t)g.rowptr.size() - 1;
    L.n = nl;
    L.nnz = g.rowptr[nl];
    L.diag.assign(nl, 0);
    for (int64_t i = 0; i < nl; ++i)
      for (int k = g.rowptr[i]; k < g.rowptr[i + 1]; ++k)
        if (g.col[k] == i) L.diag[i] = k;
    colour_classes(g, L.cptr, L.crows);
    L.rowptr = g.rowptr;
    L.col = g.col;
    if (nl <= coarse_max || level >= 15) break;
    std::vector<int32_t> agg, mptr, mem;
    const int64_t na = pairwise ? aggregate_pairs(g, agg) : aggregate(g, agg);
    if (na > (nl * 9) / 10) break;  // aggregation no longer coarsens
    HostGraph gc;
    coarsen_graph(g, agg, na, mptr, mem, gc);
    // fine entries of every coarse entry
    const int64_t nnzc = gc.rowptr[na];
    std::vector<int32_t> cmap(L.nnz), gptr(nnzc + 1, 0), gsrc(L.nnz);
    for (int64_t i = 0; i < nl; ++i) {
      const int32_t I = agg[i];
      const int32_t* b0 = gc.col.data() + gc.rowptr[I];
      const int32_t* b1 = gc.col.data() + gc.rowptr[I + 1];
      for (int k = g.rowptr[i]; k < g.rowptr[i + 1]; ++k) {
        const int32_t J = agg[g.col[k]];
        cmap[k] = (int32_t)((std::lower_bound(b0, b1, J) - gc.col.data()));
        ++gptr[cmap[k] + 1];
      }
    }
    for (int64_t k = 0; k < nnzc; ++k) gptr[k + 1] += gptr[k];
    {
      std::vector<int32_t> fill(gptr.begin(), gptr.end() - 1);
      for (int64_t k = 0; k < L.nnz; ++k) gsrc[fill[cmap[k]]++] = (int32_t)k;
    }
    L.agg = std::move(agg);
    L.mptr = std::move(mptr);
    L.mem = std::move(mem);
    L.gptr = std::move(gptr);
    L.gsrc = std::move(gsrc);
    g = std::move(gc);
  }
}

}  // namespace

hipError_t precond_create(int64_t n, int64_t ne, const int32_t* tets_dev, int coarse_max,
                          int pairwise, Precond** out) {
  *out = nullptr;
  std::vector<int32_t> T(4 * ne);
  hipError_t e = hipMemcpy(T.data(), tets_dev, sizeof(int32_t) * 4 * ne, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  std::vector<HostLevel> hl;
  build_levels(n, ne, T, coarse_max, pairwise, hl);
  T.clear();
  T.shrink_to_fit();
  const int64_t nc = hl.back().n;
  // the coarsest level is inverted densely per mode: refuse a hierarchy that
  // stopped coarsening far above coarse_max (a graph of mostly isolated
  // nodes) instead of allocating (K + 1) (4 nc)^2 complex values for it
  if (nc > kMaxCoarse) return hipErrorInvalidValue;
  std::unique_ptr<Precond> pc(new Precond());
  for (auto& H : hl) {
    pc->lv.emplace_back();
    PcLevel& L = pc->lv.back();
    L.n = H.n;
    L.nnz = H.nnz;
    if ((e = upload(L.rowptr, H.rowptr)) || (e = upload(L.col, H.col)) ||
        (e = upload(L.diag, H.diag)) || (e = upload(L.crows, H.crows)))
      return e;
    L.cptr = H.cptr;
    if ((e = L.val.ensure((size_t)L.nnz * PC_NF))) return e;
    if (!H.agg.empty() &&
        ((e = upload(L.agg, H.agg)) || (e = upload(L.mptr, H.mptr)) || (e = upload(L.mem, H.mem)) ||
         (e = upload(L.gptr, H.gptr)) || (e = upload(L.gsrc, H.gsrc))))
      return e;
  }
  pc->dense_D = 4 * nc;
  if ((e = pc->flag.ensure(1))) return e;
  *out = pc.release();
  return hipSuccess;
}

namespace {

// Vectors and trigonometric table for K + 1 modes.
hipError_t ensure_modes(Precond* pc, int N, int fp32) {
  const int nm = (N - 1) / 2 + 1;
  hipError_t e;
  if (fp32)
    for (auto& L : pc->lv) {
      const size_t len = (size_t)L.n * nm * 8;
      if ((e = L.valf.ensure((size_t)L.nnz * PC_NF)) || (e = L.xf.ensure(len)) ||
          (e = L.x2f.ensure(len)) || (e = L.bf.ensure(len)) || (e = L.rf.ensure(len)))
        return e;
    }
  if (pc->nm == nm && pc->N == N) return hipSuccess;
  for (auto& L : pc->lv) {
    const size_t len = (size_t)L.n * nm * 8;
    if ((e = L.x.ensure(len)) || (e = L.x2.ensure(len)) || (e = L.b.ensure(len)) ||
        (e = L.r.ensure(len)))
      return e;
  }
  std::vector<double> cs((size_t)nm * N * 2);
  const double two_pi = 6.283185307179586476925286766559;
  for (int m = 0; m < nm; ++m)
    for (int s = 0; s < N; ++s) {
      const double th = two_pi * (double)((m * s) % N) / (double)N;
      cs[(m * N + s) * 2] = std::cos(th);
      cs[(m * N + s) * 2 + 1] = std::sin(th);
    }
  if ((e = upload(pc->cs, cs))) return e;
  const int64_t D = pc->dense_D;
  if ((e = pc->dense.ensure((size_t)nm * D * D * 2)) || (e = pc->inv.ensure((size_t)nm * D * D * 2)) ||
      (e = pc->work.ensure((size_t)nm * D * 2 * D * 2)))
    return e;
  pc->nm = nm;
  pc->N = N;
  return hipSuccess;
}

}  // namespace

hipError_t precond_setup(Precond* pc, const DevMesh& m, const Phys& p, const double* Sy,
                         double sigma, int nu, int cycles, double wj, double gamma, int smoother,
                         int wcycle, int fp32, hipStream_t st) {
  hipError_t e = ensure_modes(pc, p.N, fp32);
  if (e != hipSuccess) return e;
  pc->fp32 = fp32;
  pc->smoother = smoother;
  pc->wcycle = wcycle;
  pc->nu = nu;
  pc->cycles = cycles;
  pc->wj = wj;
  pc->gamma = gamma;
  pc->coef = {sigma, p.rho, p.omega, pc->nm};
  PcLevel& F = pc->lv[0];
  if ((e = hipMemsetAsync(F.val.p, 0, F.val.bytes(), st))) return e;
  hipLaunchKernelGGL(k_pc_assemble, dim3(nblk(m.ne)), dim3(PBLK), 0, st, m.ne, m.n, p.N, m.tets,
                     m.geo, Sy, m.dmask, F.rowptr.p, F.col.p, F.val.p, p);
  hipLaunchKernelGGL(k_pc_dirichlet, dim3(nblk(m.n)), dim3(PBLK), 0, st, m.n, m.dmask, F.diag.p,
                     F.val.p);
  for (size_t l = 0; l + 1 < pc->lv.size(); ++l) {
    PcLevel& A = pc->lv[l];
    PcLevel& B = pc->lv[l + 1];
    hipLaunchKernelGGL(k_pc_galerkin, dim3(nblk(B.nnz * PC_NFIELDS)), dim3(PBLK), 0, st, B.nnz,
                       A.gptr.p, A.gsrc.p, A.val.p, B.val.p);
  }
  if (fp32)
    for (auto& L : pc->lv) {
      const int64_t len = L.nnz * PC_NF;
      hipLaunchKernelGGL(k_pc_narrow, dim3(nblk(len)), dim3(PBLK), 0, st, len, L.val.p, L.valf.p);
    }
  PcLevel& C = pc->lv.back();
  const int64_t D = pc->dense_D;
  if ((e = hipMemsetAsync(pc->dense.p, 0, pc->dense.bytes(), st))) return e;
  hipLaunchKernelGGL(k_pc_dense, dim3(nblk(C.nnz * pc->nm)), dim3(PBLK), 0, st, C.n, C.rowptr.p,
                     C.col.p, C.val.p, pc->coef, pc->dense.p);
  if ((e = hipMemsetAsync(pc->flag.p, 0, sizeof(int), st))) return e;
  hipLaunchKernelGGL(k_pc_invert, dim3(pc->nm), dim3(PBLK), 0, st, (int)D, pc->dense.p,
                     pc->work.p, pc->inv.p, pc->flag.p);
  return hipGetLastError();
}

namespace {

// The level's vectors and coefficients in the cycle's precision.
template <typename T>
struct LevelVecs;
template <>
struct LevelVecs<double> {
  static double*& x(PcLevel& L) { return L.x.p; }
  static double*& x2(PcLevel& L) { return L.x2.p; }
  static double* b(PcLevel& L) { return L.b.p; }
  static double* r(PcLevel& L) { return L.r.p; }
  static const double* val(PcLevel& L) { return L.val.p; }
};
template <>
struct LevelVecs<float> {
  static float*& x(PcLevel& L) { return L.xf.p; }
  static float*& x2(PcLevel& L) { return L.x2f.p; }
  static float* b(PcLevel& L) { return L.bf.p; }
  static float* r(PcLevel& L) { return L.rf.p; }
  static const float* val(PcLevel& L) { return L.valf.p; }
};

// Row operation OP on one level, one lane per (node, mode).  (One lane per
// node, or per group of modes, loads each pair's fields fewer times but
// keeps fewer waves in flight; it measured slower.)
template <int OP, typename T>
void rows(const Precond* pc, const PcLevel& L, const T* val, const T* b, const T* x, T* y,
          double wj, hipStream_t st, Corr<T> cr = {nullptr, nullptr, (T)0}) {
  hipLaunchKernelGGL((k_pc_rows<OP, T, T>), dim3(nblk(L.n * pc->nm)), dim3(PBLK), 0, st, L.n,
                     L.rowptr.p, L.col.p, L.diag.p, val, pc->coef, b, x, y, wj, cr);
}

template <typename T>
hipError_t vcycle(Precond* pc, size_t l, bool zero_start, hipStream_t st) {
  using V = LevelVecs<T>;
  PcLevel& L = pc->lv[l];
  const int nm = pc->nm;
  if (l + 1 == pc->lv.size()) {
    hipLaunchKernelGGL(k_pc_dense_apply<T>, dim3(nblk(4 * L.n * nm)), dim3(PBLK), 0, st, L.n, nm,
                       pc->inv.p, V::b(L), V::x(L));
    return hipGetLastError();
  }
  Corr<T> cr{nullptr, nullptr, (T)0};
  auto sweep = [&](bool from_zero, bool reverse) {
    if (pc->smoother == 1) {
      if (from_zero)
        hipLaunchKernelGGL(k_pc_zero<T>, dim3(nblk(L.n * nm * 8)), dim3(PBLK), 0, st,
                           L.n * nm * 8, V::x(L));
      const int nc = (int)L.cptr.size() - 1;
      for (int q = 0; q < nc; ++q) {
        const int c = reverse ? nc - 1 - q : q;
        const int64_t nr = L.cptr[c + 1] - L.cptr[c];
        hipLaunchKernelGGL((k_pc_gs<T, T>), dim3(nblk(nr * nm)), dim3(PBLK), 0, st, nr,
                           L.crows.p + L.cptr[c], L.rowptr.p, L.col.p, L.diag.p, V::val(L),
                           pc->coef, V::b(L), V::x(L));
      }
      return;
    }
    rows<2, T>(pc, L, V::val(L), V::b(L), from_zero ? nullptr : V::x(L), V::x2(L), pc->wj, st,
               cr);
    std::swap(V::x(L), V::x2(L));
  };
  for (int k = 0; k < pc->nu; ++k) sweep(zero_start && k == 0, false);
  rows<1, T>(pc, L, V::val(L), V::b(L), V::x(L), V::r(L), 0.0, st);
  PcLevel& C = pc->lv[l + 1];
  hipLaunchKernelGGL(k_pc_restrict<T>, dim3(nblk(C.n * nm * 8)), dim3(PBLK), 0, st, C.n, nm,
                     L.mptr.p, L.mem.p, V::r(L), V::b(C));
  hipError_t e = vcycle<T>(pc, l + 1, true, st);
  if (e != hipSuccess) return e;
  if (pc->wcycle && l + 2 < pc->lv.size()) {
    e = vcycle<T>(pc, l + 1, false, st);
    if (e != hipSuccess) return e;
  }
  if (pc->smoother == 1) {
    hipLaunchKernelGGL(k_pc_prolong<T>, dim3(nblk(L.n * nm * 8)), dim3(PBLK), 0, st, L.n, nm,
                       L.agg.p, V::x(C), V::x(L), pc->gamma);
    for (int k = 0; k < pc->nu; ++k) sweep(false, true);
  } else {
    // the first post-smoothing sweep reads x + gamma P xc (the prolongation)
    cr = {V::x(C), L.agg.p, (T)pc->gamma};
    sweep(false, true);
    cr = {nullptr, nullptr, (T)0};
    for (int k = 1; k < pc->nu; ++k) sweep(false, true);
  }
  return hipGetLastError();
}

template <typename T, typename TQ, typename TZ>
hipError_t apply_in(Precond* pc, int64_t n, const TQ* q, int in_ch, TZ* z, hipStream_t st) {
  using V = LevelVecs<T>;
  const int nm = pc->nm, N = pc->N;
  PcLevel& F = pc->lv[0];
  launch_to_modes<TQ, T>(n, N, nm, q, in_ch, pc->cs.p, V::b(F), st);
  for (int c = 0; c < pc->cycles; ++c) {
    hipError_t e = vcycle<T>(pc, 0, c == 0, st);
    if (e != hipSuccess) return e;
  }
  launch_from_modes<T, TZ>(n, N, nm, V::x(F), pc->cs.p, z, st);
  return hipGetLastError();
}

}  // namespace

template <typename TQ, typename TZ>
hipError_t precond_apply(Precond* pc, int64_t n, const TQ* q, int in_ch, TZ* z, hipStream_t st) {
  return pc->fp32 ? apply_in<float>(pc, n, q, in_ch, z, st)
                  : apply_in<double>(pc, n, q, in_ch, z, st);
}

template <typename TQ, typename TZ>
hipError_t precond_matvec(Precond* pc, int64_t n, const TQ* q, int in_ch, TZ* z, hipStream_t st) {
  const int nm = pc->nm, N = pc->N;
  PcLevel& F = pc->lv[0];
  launch_to_modes<TQ, double>(n, N, nm, q, in_ch, pc->cs.p, F.b.p, st);
  hipLaunchKernelGGL((k_pc_rows<0, double, double>), dim3(nblk(n * nm)), dim3(PBLK), 0, st, n,
                     F.rowptr.p, F.col.p, F.diag.p, F.val.p, pc->coef, nullptr, F.b.p, F.x.p, 0.0,
                     Corr<double>{nullptr, nullptr, 0.0});
  launch_from_modes<double, TZ>(n, N, nm, F.x.p, pc->cs.p, z, st);
  return hipGetLastError();
}

hipError_t precond_singular(Precond* pc, int* flag_host, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(flag_host, pc->flag.p, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

template hipError_t precond_apply<double, double>(Precond*, int64_t, const double*, int,
                                                  double*, hipStream_t);
template hipError_t precond_apply<float, double>(Precond*, int64_t, const float*, int, double*,
                                                 hipStream_t);
template hipError_t precond_matvec<double, double>(Precond*, int64_t, const double*, int,
                                                   double*, hipStream_t);

}  // namespace hb

extern "C" int hb_precond_hierarchy(int64_t n, int64_t ne, const int32_t* tets, int32_t coarse_max,
                                    int32_t aggregation, int32_t max_levels, int64_t* sizes,
                                    int32_t* n_levels, int32_t* agg0, int32_t* colour0) {
  auto fail = [](const char* msg) {
    hb::set_last_error(msg);
    return (int)HB_ERR_ARG;
  };
  if (n < 1 || ne < 1 || !tets || !sizes || !n_levels || max_levels < 1)
    return fail("bad argument");
  if (n > INT32_MAX || coarse_max < 1 || coarse_max > 256 || (aggregation != 0 && aggregation != 1))
    return fail("bad hierarchy options");
  std::vector<int32_t> soa(4 * (size_t)ne);
  for (int64_t t = 0; t < ne; ++t)
    for (int A = 0; A < 4; ++A) {
      const int32_t v = tets[4 * t + A];
      if (v < 0 || v >= n) return fail("tetrahedron node index out of range");
      soa[(size_t)A * ne + t] = v;
    }
  std::vector<hb::HostLevel> hl;
  hb::build_levels(n, ne, soa, coarse_max, aggregation == 0, hl);
  *n_levels = (int32_t)hl.size();
  for (int32_t l = 0; l < max_levels && l < (int32_t)hl.size(); ++l) sizes[l] = hl[l].n;
  if (agg0)
    for (int64_t i = 0; i < n; ++i) agg0[i] = hl[0].agg.empty() ? -1 : hl[0].agg[i];
  if (colour0) {
    const auto& L = hl[0];
    for (size_t c = 0; c + 1 < L.cptr.size(); ++c)
      for (int64_t k = L.cptr[c]; k < L.cptr[c + 1]; ++k) colour0[L.crows[k]] = (int32_t)c;
  }
  return HB_OK;
}
