// HIP kernels of the harmonic-balance GLS Navier-Stokes operator for gfx950.
//
// The operator (Jia & Esmaily, arXiv 2411.14315, Section 2.3, eq. Rmc) is
// pointwise in time except for the time-coupling matrix H (Section 2.1,
// eq. NS-harm).  The hot path is split accordingly:
//
//   node tiles   modal <-> time-sample transforms and H products, one small
//                dense N x N contraction per node and field, staged through
//                LDS so that every global access is a contiguous run (FP64
//                on the vector ALU; the FP32 paths run them as 32 x 32 tiles
//                on the matrix cores with split-BF16 operands);
//   elements     one quad of four lanes per (tetrahedron, sample) for the
//                residual and exact Jacobian-vector kernels (lane A holds
//                node A and quadrature point A; element sums and the row
//                scatter go through quad shuffles, then 7 FP64 hardware
//                atomics per lane); one lane per (tetrahedron, sample) for
//                the paper tangent and the Jacobi diagonal; workgroups are
//                mapped so that each XCD (own L2) walks a contiguous range
//                of elements;
//   faces        one lane per (outlet triangle, sample): traction,
//                resistance and backflow terms.
//
// Layouts: modal arrays [f][m][node]; sample buffers node-major
// [node][channel][sample], so the N lanes of one element read N contiguous
// doubles per node and channel.
#include "hb_internal.h"

#include <atomic>
#include <type_traits>

namespace hb {

namespace {

constexpr int BLK = 256;
constexpr int TN = 32;  // nodes per transform tile
// 4-point degree-2 tetrahedron rule: barycentric (a, b, b, b) and permutations.
constexpr double QA = 0.58541019662496845446137605030969;
constexpr double QB = 0.13819660112501051517954131656344;
constexpr double TRI_A = 2.0 / 3.0, TRI_B = 1.0 / 6.0;

// Map the hardware workgroup id to a logical one so that the XCD that
// receives workgroups b, b+8, b+16, ... processes one contiguous range.
__device__ __forceinline__ int64_t xcd_block(int64_t nlogical) {
  const int64_t g = gridDim.x;
  const int64_t per = g >> 3;
  const int64_t b = blockIdx.x;
  const int64_t lb = (b & 7) * per + (b >> 3);
  return lb < nlogical ? lb : -1;
}

inline unsigned xcd_grid(int64_t nlogical) {
  int64_t g = (nlogical + 7) & ~int64_t(7);
  return (unsigned)g;
}

__device__ __forceinline__ void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }

template <typename R>
struct GeoT {
  R g[4][3];
  R V, x00, x01, x02, x11, x12, x22, xixi;
};
using Geo = GeoT<double>;

template <typename R>
__device__ __forceinline__ void load_geo(const double* __restrict__ geo, int64_t ne, int64_t t,
                                         GeoT<R>& G) {
#pragma unroll
  for (int A = 1; A < 4; ++A)
#pragma unroll
    for (int i = 0; i < 3; ++i) G.g[A][i] = geo[(GEO_G1 + 3 * (A - 1) + i) * ne + t];
#pragma unroll
  for (int i = 0; i < 3; ++i) G.g[0][i] = -(G.g[1][i] + G.g[2][i] + G.g[3][i]);
  G.V = geo[GEO_V * ne + t];
  G.x00 = geo[GEO_XI00 * ne + t];
  G.x01 = geo[GEO_XI01 * ne + t];
  G.x02 = geo[GEO_XI02 * ne + t];
  G.x11 = geo[GEO_XI11 * ne + t];
  G.x12 = geo[GEO_XI12 * ne + t];
  G.x22 = geo[GEO_XI22 * ne + t];
  G.xixi = geo[GEO_XIXI * ne + t];
}

// tau = 1 / sqrt(x), x > 0: the hardware reciprocal-square-root estimate
// refined by Newton steps y <- y + y (1 - x y^2) / 2 (two in FP64, one in
// FP32), each of which doubles the number of correct bits.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double r = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, r, y);
  }
  return y;
}
__device__ __forceinline__ float rsqrt_nr(float x) {
  const float y = __builtin_amdgcn_rsqf(x);
  return fmaf(0.5f * y, fmaf(-x * y, y, 1.0f), y);
}

template <typename R>
__device__ __forceinline__ void xi_mul(const GeoT<R>& G, const R u[3], R o[3]) {
  o[0] = G.x00 * u[0] + G.x01 * u[1] + G.x02 * u[2];
  o[1] = G.x01 * u[0] + G.x11 * u[1] + G.x12 * u[2];
  o[2] = G.x02 * u[0] + G.x12 * u[1] + G.x22 * u[2];
}

// ------------------------------------------------------------ MFMA tiles

// Time-axis contractions of the FP32 paths on the matrix cores: a 32 x 32
// output tile C = A B (A: N x N time table or H, B: N x 32 node columns)
// per wavefront, N padded to 32 rows and to a multiple of 8 in k.  Operands
// are split into BF16 high and low parts, x = hi + lo, and three BF16 MFMAs
// per k-step (hi.hi + hi.lo + lo.hi) accumulate in FP32, which keeps about
// 16 significant bits of each product (split-BF16).
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ inline short bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ inline float bf16_val(short b) { return __uint_as_float((uint32_t)(uint16_t)b << 16); }

// Lane layout of v_mfma_f32_32x32x8 (wavefront of 64): lane l supplies
// A[l % 32][k0 + 4 (l / 32) + t] and B[k0 + 4 (l / 32) + t][l % 32], t < 4,
// and holds C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] in register r < 16.
// FA(i, k) and FB(k, j) return 0 outside the matrices.
template <class FA, class FB>
__device__ inline f32x16 mfma_tile_split(int N, FA A, FB B) {
  const int lane = threadIdx.x & 63;
  const int ij = lane & 31, kq = (lane >> 5) * 4;
  f32x16 c = {};
  for (int k0 = 0; k0 < N; k0 += 8) {
    bf16x4 ah, alo, bh, blo;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = k0 + kq + t;
      const float a = (float)A(ij, k);
      const float b = (float)B(k, ij);
      const short a1 = bf16_rne(a), b1 = bf16_rne(b);
      ah[t] = a1;
      bh[t] = b1;
      alo[t] = bf16_rne(a - bf16_val(a1));
      blo[t] = bf16_rne(b - bf16_val(b1));
    }
    c = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, blo, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(alo, bh, c, 0, 0, 0);
  }
  return c;
}
// row of register r of this lane in the C tile (the column is lane % 32)
__device__ inline int mfma_row(int r) { return 8 * (r >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (r & 3); }

// ------------------------------------------------------------ node tiles

// Modal Y[f][m][a] -> samples S[a][c][s]: c = 0..3 values, 4..6 time
// derivative of the velocity (H u).  Dirichlet velocity entries are replaced
// by the boundary data (zero_dirichlet = 0) or by zero (= 1).  Optionally
// clears the element accumulator of the tile and a short vector.
template <typename TI, typename TO, int TL>
__global__ void __launch_bounds__(BLK)
k_modal_to_samples(int64_t n, int N, const TI* __restrict__ Y, const double* __restrict__ dir,
                   const uint8_t* __restrict__ dmask, int zero_dirichlet,
                   const double* __restrict__ tab, TO* __restrict__ S,
                   TO* __restrict__ acc, double* __restrict__ qz, int nq) {
  extern __shared__ double sm[];
  double* sY = sm;              // [4][N][TL]
  double* sB = sY + 4 * N * TL; // Binv [s][m]
  double* sD = sB + N * N;      // Bder [s][m]
  const int64_t a0 = (int64_t)blockIdx.x * TL;
  const int tn = (int)min<int64_t>(TL, n - a0);
  const int NN = N * N;
  for (int i = threadIdx.x; i < NN; i += BLK) {
    sB[i] = tab[TAB_BINV * NN + i];
    sD[i] = tab[TAB_BDER * NN + i];
  }
  for (int i = threadIdx.x; i < 4 * N * TL; i += BLK) {
    const int al = i % TL;
    const int fm = i / TL;
    double v = 0.0;
    if (al < tn) {
      const int64_t a = a0 + al;
      v = (double)Y[(int64_t)fm * n + a];
      if (fm < 3 * N && dmask[a]) v = zero_dirichlet ? 0.0 : dir[(int64_t)fm * n + a];
    }
    sY[i] = v;
  }
  if (acc) {
    TO* ap = acc + a0 * NCH * N;
    for (int i = threadIdx.x; i < tn * NCH * N; i += BLK) ap[i] = TO(0);
  }
  if (qz && blockIdx.x == 0)
    for (int i = threadIdx.x; i < nq; i += BLK) qz[i] = 0.0;
  __syncthreads();
  if constexpr (std::is_same<TO, float>::value) {
    if (N <= 32 && TL == 32) {
      // 7 tiles: Binv Y_f (f < 4) and Bder Y_f (f < 3), one per wavefront
      const int lane = threadIdx.x & 63;
      for (int tile = threadIdx.x >> 6; tile < 7; tile += BLK / 64) {
        const int f = tile < 4 ? tile : tile - 4;
        const double* T = tile < 4 ? sB : sD;
        const f32x16 c = mfma_tile_split(
            N, [&](int i, int k) { return (i < N && k < N) ? T[i * N + k] : 0.0; },
            [&](int k, int j) { return k < N ? sY[(f * N + k) * TL + j] : 0.0; });
        const int al = lane & 31;
        if (al < tn) {
          TO* out = S + (a0 + al) * NCH * N + tile * N;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int sr = mfma_row(r);
            if (sr < N) out[sr] = c[r];
          }
        }
      }
      return;
    }
  }
  for (int it = threadIdx.x; it < tn * N; it += BLK) {
    const int al = it / N;
    const int s = it - al * N;
    double o[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int m = 0; m < N; ++m) {
      const double b = sB[s * N + m];
      const double d = sD[s * N + m];
#pragma unroll
      for (int f = 0; f < 4; ++f) o[f] += b * sY[(f * N + m) * TL + al];
#pragma unroll
      for (int f = 0; f < 3; ++f) o[4 + f] += d * sY[(f * N + m) * TL + al];
    }
    TO* out = S + (a0 + al) * NCH * N + s;
#pragma unroll
    for (int c = 0; c < 7; ++c) out[c * N] = (TO)o[c];
  }
}

// Samples acc[a][c][s] -> modal R[f][m][a].  Momentum rows receive -H z,
// i.e. -FwdD applied to the z channels (use_z), and are zeroed at Dirichlet
// nodes when zero_dir_rows.
template <typename TA, typename TO, int TL>
__global__ void __launch_bounds__(BLK)
k_samples_to_modal(int64_t n, int N, const TA* __restrict__ acc, int use_z, int zero_dir_rows,
                   int in_ch, const uint8_t* __restrict__ dmask, const double* __restrict__ tab,
                   TO* __restrict__ R) {
  extern __shared__ double sm[];
  const int CN = in_ch * N;
  double* sA = sm;              // [TL][in_ch][N]
  double* sF = sA + TL * CN;    // Fwd [m][s]
  double* sG = sF + N * N;      // FwdD [m][s]
  const int64_t a0 = (int64_t)blockIdx.x * TL;
  const int tn = (int)min<int64_t>(TL, n - a0);
  const int NN = N * N;
  for (int i = threadIdx.x; i < NN; i += BLK) {
    sF[i] = tab[TAB_FWD * NN + i];
    sG[i] = tab[TAB_FWDD * NN + i];
  }
  const TA* ap = acc + a0 * CN;
  for (int i = threadIdx.x; i < tn * CN; i += BLK) sA[i] = (double)ap[i];
  __syncthreads();
  if constexpr (std::is_same<TO, float>::value) {
    if (N <= 32 && TL == 32) {
      // 4 tiles (one per field): Fwd A_f, minus FwdD z_f on momentum rows
      const int lane = threadIdx.x & 63;
      const int f = threadIdx.x >> 6;  // BLK / 64 == 4 wavefronts, one field each
      const bool wz = f < 3 && use_z;
      const int K2 = wz ? 2 * N : N;   // [Fwd | -FwdD] against [A_f ; z_f]
      const f32x16 c = mfma_tile_split(
          K2,
          [&](int i, int k) {
            if (i >= N || k >= K2) return 0.0;
            return k < N ? sF[i * N + k] : -sG[i * N + (k - N)];
          },
          [&](int k, int j) {
            if (j >= tn || k >= K2) return 0.0;
            const double* row = sA + j * CN;
            return k < N ? row[f * N + k] : row[(4 + f) * N + (k - N)];
          });
      const int al = lane & 31;
      if (al < tn) {
        const bool zero = f < 3 && zero_dir_rows && dmask[a0 + al];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = mfma_row(r);
          if (m < N) R[(int64_t)(f * N + m) * n + a0 + al] = zero ? TO(0) : (TO)c[r];
        }
      }
      return;
    }
  }
  for (int it = threadIdx.x; it < 4 * N * tn; it += BLK) {
    const int al = it % tn;
    const int fm = it / tn;
    const int f = fm / N;
    const int m = fm - f * N;
    const double* row = sA + al * CN;
    double v = 0.0;
    for (int s = 0; s < N; ++s) v += sF[m * N + s] * row[f * N + s];
    if (f < 3) {
      if (use_z)
        for (int s = 0; s < N; ++s) v -= sG[m * N + s] * row[(4 + f) * N + s];
      if (zero_dir_rows && dmask[a0 + al]) v = 0.0;
    }
    R[(int64_t)fm * n + a0 + al] = (TO)v;
  }
}

// Sample-space direction: v = P^-1 q with P^-1 the pointwise inverse
// diagonal dinv, or for velocity the per-node time blocks binv (pressure
// still dinv); velocity entries of Dirichlet nodes zeroed if zero_dirichlet.
// Then Sv[a][0..3] = v and Sv[a][4..6] = H v.  q may alias Sv when
// in_ch == NCH (state update in place).
template <typename TQ, typename TS>
__global__ void __launch_bounds__(BLK)
k_prepare(int64_t n, int N, const TQ* q, int in_ch, const double* __restrict__ dinv,
          const double* __restrict__ binv, int zero_dirichlet, const uint8_t* __restrict__ dmask,
          const double* __restrict__ tab, TS* Sv, TS* __restrict__ acc,
          double* __restrict__ qz, int nq) {
  extern __shared__ double sm[];
  double* sV = sm;              // [TN][4][N]
  double* sH = sV + TN * 4 * N; // H [s][k]
  double* sQ = sH + N * N;      // [TN][3][N] raw velocity (block path only)
  const int64_t a0 = (int64_t)blockIdx.x * TN;
  const int tn = (int)min<int64_t>(TN, n - a0);
  const int NN = N * N;
  for (int i = threadIdx.x; i < NN; i += BLK) sH[i] = tab[TAB_H * NN + i];
  for (int i = threadIdx.x; i < tn * 4 * N; i += BLK) {
    const int al = i / (4 * N);
    const int r = i - al * 4 * N;
    const int c = r / N;
    const int s = r - c * N;
    const int64_t a = a0 + al;
    double v = (double)q[(a * in_ch + c) * N + s];
    if (binv && c < 3) {
      sQ[(al * 3 + c) * N + s] = v;
    } else if (dinv) {
      v *= dinv[(a * 2 + (c < 3 ? 0 : 1)) * N + s];
    }
    if (zero_dirichlet && c < 3 && dmask[a]) v = 0.0;
    sV[i] = v;
  }
  if (acc) {
    TS* ap = acc + a0 * NCH * N;
    for (int i = threadIdx.x; i < tn * NCH * N; i += BLK) ap[i] = TS(0);
  }
  if (qz && blockIdx.x == 0)
    for (int i = threadIdx.x; i < nq; i += BLK) qz[i] = 0.0;
  __syncthreads();
  if (binv) {
    for (int it = threadIdx.x; it < tn * N; it += BLK) {
      const int al = it / N;
      const int s = it - al * N;
      const int64_t a = a0 + al;
      if (zero_dirichlet && dmask[a]) continue;
      const double* row = binv + (a * N + s) * N;
      double v0 = 0.0, v1 = 0.0, v2 = 0.0;
      const double* q3 = sQ + al * 3 * N;
      for (int k = 0; k < N; ++k) {
        const double b = row[k];
        v0 += b * q3[k];
        v1 += b * q3[N + k];
        v2 += b * q3[2 * N + k];
      }
      double* v = sV + al * 4 * N;
      v[s] = v0;
      v[N + s] = v1;
      v[2 * N + s] = v2;
    }
    __syncthreads();
  }
  if constexpr (std::is_same<TS, float>::value) {
    if (N <= 32 && TN == 32) {
      for (int it = threadIdx.x; it < tn * 4 * N; it += BLK) {
        const int al = it / (4 * N);
        const int r = it - al * 4 * N;
        Sv[(a0 + al) * NCH * N + r] = (TS)sV[it];
      }
      // H v for the three velocity channels, one tile per wavefront
      const int lane = threadIdx.x & 63;
      const int c = threadIdx.x >> 6;
      if (c < 3) {
        const f32x16 hv = mfma_tile_split(
            N, [&](int i, int k) { return (i < N && k < N) ? sH[i * N + k] : 0.0; },
            [&](int k, int j) { return (k < N && j < tn) ? sV[j * 4 * N + c * N + k] : 0.0; });
        const int al = lane & 31;
        if (al < tn) {
          TS* out = Sv + (a0 + al) * NCH * N + (4 + c) * N;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int sr = mfma_row(r);
            if (sr < N) out[sr] = hv[r];
          }
        }
      }
      return;
    }
  }
  for (int it = threadIdx.x; it < tn * N; it += BLK) {
    const int al = it / N;
    const int s = it - al * N;
    const double* v = sV + al * 4 * N;
    double h0 = 0.0, h1 = 0.0, h2 = 0.0;
    for (int k = 0; k < N; ++k) {
      const double hk = sH[s * N + k];
      h0 += hk * v[k];
      h1 += hk * v[N + k];
      h2 += hk * v[2 * N + k];
    }
    TS* out = Sv + (a0 + al) * NCH * N + s;
    out[0] = (TS)v[s];
    out[N] = (TS)v[N + s];
    out[2 * N] = (TS)v[2 * N + s];
    out[3 * N] = (TS)v[3 * N + s];
    out[4 * N] = (TS)h0;
    out[5 * N] = (TS)h1;
    out[6 * N] = (TS)h2;
  }
}

// The velocity block of the exact Jacobian's nodal diagonal in time,
//   B = diag(K_AA) + rho M_AA H + diag(X_AA) H - H diag(X_AA) - rho H diag(T_AA) H
// (Galerkin time term, and the stabilisation's time terms: the test
// function's -H N_A against tau L, with L's rho H u and rho u.grad u, and
// the streamline test against tau rho H u), inverted by Gauss-Jordan
// elimination without pivoting (the symmetric part of B is diag(K_AA) +
// rho H^T diag(T_AA) H, positive).
//
// One wavefront per workgroup handles P = floor(64 / N) consecutive nodes
// (3 at N = 21), each block in LDS.  Building B spreads the P N^2 entries
// over all lanes; in the elimination lane (q, j) owns column j of node q's
// block.  Within a wavefront, LDS accesses are ordered by program order, so
// the elimination needs no barrier: in every row chunk all lanes read the
// pivot column before the pivot column's owner writes it.  Requires
// N <= 64.  Identity at Dirichlet nodes.  dg has 4 channels (K, L, T, X),
// node-major, so the P nodes' rows are one contiguous range.
constexpr int FACT_CHUNK = 4;
__global__ void __launch_bounds__(64)
k_block_factor(int64_t n, int N, int P, const double* __restrict__ dg,
               const double* __restrict__ mass, double rho, const double* __restrict__ tab,
               const uint8_t* __restrict__ dmask, double* __restrict__ binv) {
  extern __shared__ double sm[];
  const int NN = N * N;
  double* sH = sm;                  // [N][N]
  double* sD = sH + NN;             // [P][4][N]  K, L, T, X
  double* sB = sD + P * 4 * N;      // [P][N][N]
  const int lane = threadIdx.x;
  const int64_t a0 = (int64_t)blockIdx.x * P;
  const int np = (int)min<int64_t>(P, n - a0);
  for (int i = lane; i < NN; i += 64) sH[i] = tab[TAB_H * NN + i];
  const double* src = dg + a0 * 4 * N;
  for (int i = lane; i < np * 4 * N; i += 64) sD[i] = src[i];
  __syncthreads();

  // B entries, e = (q, s, j)
  for (int e = lane; e < np * NN; e += 64) {
    const int q = e / NN;
    const int r = e - q * NN;
    const int sr = r / N;
    const int j = r - sr * N;
    const int64_t a = a0 + q;
    double v;
    if (dmask[a]) {
      v = (sr == j) ? 1.0 : 0.0;
    } else {
      const double* Kd = sD + q * 4 * N;
      const double* Td = Kd + 2 * N;
      const double* Xd = Kd + 3 * N;
      const double hsj = sH[sr * N + j];
      v = (rho * mass[a] + Xd[sr]) * hsj - hsj * Xd[j];
      double h2 = 0.0;
      for (int t = 0; t < N; ++t) h2 += sH[sr * N + t] * Td[t] * sH[t * N + j];
      v -= rho * h2;
      if (sr == j) v += Kd[sr];
    }
    sB[e] = v;
  }
  __syncthreads();

  // Gauss-Jordan inversion in place; lane (q, j)
  const int q = lane / N;
  const int j = lane - q * N;
  const bool act = q < np;
  double* B = sB + (act ? q : 0) * NN;
  for (int kp = 0; kp < N; ++kp) {
    if (act) {
      const double ip = 1.0 / B[kp * N + kp];
      const double rk = (j == kp) ? ip : B[kp * N + j] * ip;
      for (int i0 = 0; i0 < N; i0 += FACT_CHUNK) {
        double f[FACT_CHUNK], b[FACT_CHUNK];
#pragma unroll
        for (int c = 0; c < FACT_CHUNK; ++c) {
          const int i = i0 + c;
          f[c] = i < N ? B[i * N + kp] : 0.0;
          b[c] = i < N ? B[i * N + j] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < FACT_CHUNK; ++c) {
          const int i = i0 + c;
          if (i < N) B[i * N + j] = (i == kp) ? rk : (j == kp ? 0.0 : b[c]) - f[c] * rk;
        }
      }
    }
  }
  __syncthreads();
  double* out = binv + a0 * NN;
  for (int e = lane; e < np * NN; e += 64) out[e] = sB[e];
}

// Sample-space rows: out[a][i][s] = acc r^m_i - (H z_i) (use_z), out[a][3] =
// r^c; Dirichlet momentum rows take id_rows (identity) or zero.
template <typename TA, typename TO>
__global__ void __launch_bounds__(BLK)
k_finish(int64_t n, int N, const TA* __restrict__ acc, int use_z,
         const uint8_t* __restrict__ dmask, const double* __restrict__ tab,
         const TO* __restrict__ id_rows, TO* __restrict__ out) {
  extern __shared__ double sm[];
  double* sA = sm;                 // [TN][7][N]
  double* sH = sA + TN * NCH * N;
  const int64_t a0 = (int64_t)blockIdx.x * TN;
  const int tn = (int)min<int64_t>(TN, n - a0);
  const int NN = N * N;
  for (int i = threadIdx.x; i < NN; i += BLK) sH[i] = tab[TAB_H * NN + i];
  const TA* ap = acc + a0 * NCH * N;
  for (int i = threadIdx.x; i < tn * NCH * N; i += BLK) sA[i] = (double)ap[i];
  __syncthreads();
  if constexpr (std::is_same<TO, float>::value) {
    if (N <= 32 && TN == 32 && use_z) {
      // momentum rows: acc_c - H z_c on the matrix cores (one channel per
      // wavefront); the pressure rows are copied
      const int lane = threadIdx.x & 63;
      const int c = threadIdx.x >> 6;
      if (c < 3) {
        const f32x16 hz = mfma_tile_split(
            N, [&](int i, int k) { return (i < N && k < N) ? sH[i * N + k] : 0.0; },
            [&](int k, int j) {
              return (k < N && j < tn) ? sA[j * NCH * N + (4 + c) * N + k] : 0.0;
            });
        const int al = lane & 31;
        if (al < tn) {
          const int64_t a = a0 + al;
          const double* row = sA + al * NCH * N;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int sr = mfma_row(r);
            if (sr < N) {
              const double v = dmask[a] ? (id_rows ? (double)id_rows[(a * 4 + c) * N + sr] : 0.0)
                                         : row[c * N + sr] - (double)hz[r];
              out[(a * 4 + c) * N + sr] = (TO)v;
            }
          }
        }
      } else {
        for (int it = lane; it < tn * N; it += 64) {
          const int al = it / N;
          const int sr = it - al * N;
          out[((a0 + al) * 4 + 3) * N + sr] = (TO)sA[al * NCH * N + 3 * N + sr];
        }
      }
      return;
    }
  }
  for (int it = threadIdx.x; it < tn * 4 * N; it += BLK) {
    const int al = it / (4 * N);
    const int r = it - al * 4 * N;
    const int c = r / N;
    const int s = r - c * N;
    const int64_t a = a0 + al;
    const double* row = sA + al * NCH * N;
    double v = row[c * N + s];
    if (c < 3) {
      if (use_z) {
        const double* z = row + (4 + c) * N;
        for (int k = 0; k < N; ++k) v -= sH[s * N + k] * z[k];
      }
      if (dmask[a]) v = id_rows ? (double)id_rows[(a * 4 + c) * N + s] : 0.0;
    }
    out[(a * 4 + c) * N + s] = (TO)v;
  }
}

// ------------------------------------------------------------- elements

// Scatter of one element-sample's 4 x 7 rows.
__device__ __forceinline__ void scatter_rows(double* __restrict__ acc, const int64_t base[4],
                                             int N, const double rm[4][3], const double rc[4],
                                             const double z[4][3], bool with_z) {
#pragma unroll
  for (int A = 0; A < 4; ++A) {
    double* p = acc + base[A];
    atomic_add(p, rm[A][0]);
    atomic_add(p + N, rm[A][1]);
    atomic_add(p + 2 * N, rm[A][2]);
    atomic_add(p + 3 * N, rc[A]);
    if (with_z) {
      atomic_add(p + 4 * N, z[A][0]);
      atomic_add(p + 5 * N, z[A][1]);
      atomic_add(p + 6 * N, z[A][2]);
    }
  }
}

// Quad-lane element kernels: one (tetrahedron, sample) is spread over the
// four lanes of a quad, lane A holding node A and quadrature point A of the
// 4-point rule (its barycentric weights are QA at node A and QB at the
// others).  Element-constant sums are all-reduced across the quad; each
// lane forms its quadrature point's contributions to the rows of all four
// nodes; a reduce-scatter across the quad leaves lane A with node A's seven
// rows, which it adds to the accumulator with seven atomics.

// Exchange with the lane whose index differs in bit 0 (CTRL = 0xB1, quad
// permutation [1,0,3,2]) or bit 1 (CTRL = 0x4E, [2,3,0,1]) through DPP
// moves, which stay in the vector ALU (no LDS crossbar traffic).  All four
// lanes of a quad are always active together.
template <int CTRL>
__device__ __forceinline__ double quad_swap(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float quad_swap(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
constexpr int XOR1 = 0xB1, XOR2 = 0x4E, XOR3 = 0x1B;  // quad_perm [1,0,3,2], [2,3,0,1], [3,2,1,0]

template <typename R>
__device__ __forceinline__ R quad_sum(R v) {
  v += quad_swap<XOR1>(v);
  v += quad_swap<XOR2>(v);
  return v;
}

// Relative order: lane A holds ck[k][c], its contribution to node A ^ k.
// Lane A ^ k's entry k is its contribution to node A, so one exchange per k
// collects node A's rows without lane-dependent selects.
template <typename R>
__device__ __forceinline__ void quad_gather_rows(R ck[4][NCH], R out[NCH]) {
#pragma unroll
  for (int c = 0; c < NCH; ++c)
    out[c] = ck[0][c] + quad_swap<XOR1>(ck[1][c]) + quad_swap<XOR2>(ck[2][c]) +
             quad_swap<XOR3>(ck[3][c]);
}

// Element geometry as seen by lane A of a quad: g[k] = grad N_(A ^ k) (its
// own gradient loaded, the others exchanged within the quad), the volume
// and xi.
template <typename R>
__device__ __forceinline__ void load_geo_lane(const double* __restrict__ geo, int64_t ne,
                                              int64_t t, int A, GeoT<R>& G) {
  const int row = A == 0 ? GEO_G0 : GEO_G1 + 3 * (A - 1);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    G.g[0][i] = (R)geo[(row + i) * ne + t];
    G.g[1][i] = quad_swap<XOR1>(G.g[0][i]);
    G.g[2][i] = quad_swap<XOR2>(G.g[0][i]);
    G.g[3][i] = quad_swap<XOR3>(G.g[0][i]);
  }
  G.V = geo[GEO_V * ne + t];
  G.x00 = geo[GEO_XI00 * ne + t];
  G.x01 = geo[GEO_XI01 * ne + t];
  G.x02 = geo[GEO_XI02 * ne + t];
  G.x11 = geo[GEO_XI11 * ne + t];
  G.x12 = geo[GEO_XI12 * ne + t];
  G.x22 = geo[GEO_XI22 * ne + t];
  G.xixi = geo[GEO_XIXI * ne + t];
}

// Residual of eq. Rmc for one (tetrahedron, sample):
//   r^m_Ai += int N_A rho (Hu_i + u.grad u_i) + (u.grad N_A) tau L_i
//             + mu grad N_A . grad u_i - d_i N_A p
//   z_Ai   += int N_A tau L_i           (receives -H per node afterwards)
//   r^c_A  += int N_A div u + (1/rho) d_i N_A tau L_i
// with L_i = rho (Hu_i + u.grad u_i) + d_i p and tau from eq. tau.
// Lane body: this lane's node row values (7 channels) for element t, sample
// s, node/quadrature index A; returns the node's accumulator offset.
__device__ __forceinline__ int64_t residual_lane(const DevMesh& m, const Phys& p,
                                                 const double* __restrict__ S, int64_t t, int s,
                                                 int A, double res[NCH]) {
  const int N = p.N;
  Geo G;  // G.g[k] = grad N_(A ^ k)
  load_geo_lane(m.geo, m.ne, t, A, G);
  const double* gA = G.g[0];
  const int64_t base = (int64_t)m.tets[A * m.ne + t] * NCH * N + s;
  const double* q = S + base;
  double u[3], hu[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    u[i] = q[i * N];
    hu[i] = q[(4 + i) * N];
  }
  const double pr = q[3 * N];
  double Gm[3][3], gp[3], uq[3], hq[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) Gm[i][j] = quad_sum(u[i] * gA[j]);
    gp[i] = quad_sum(pr * gA[i]);
    uq[i] = QB * quad_sum(u[i]) + (QA - QB) * u[i];
    hq[i] = QB * quad_sum(hu[i]) + (QA - QB) * hu[i];
  }
  const double pbar = 0.25 * quad_sum(pr);
  const double rho = p.rho;
  const double w = 0.25 * G.V;
  double adv[3], xu[3], sv[3], gal[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) adv[i] = uq[0] * Gm[i][0] + uq[1] * Gm[i][1] + uq[2] * Gm[i][2];
  xi_mul(G, uq, xu);
  const double tau =
      rsqrt_nr(uq[0] * xu[0] + uq[1] * xu[1] + uq[2] * xu[2] + p.C_I * p.nu * p.nu * G.xixi +
               p.tau_add);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gal[i] = rho * (hq[i] + adv[i]);
    sv[i] = tau * (gal[i] + gp[i]);
  }
  double cr[4][NCH];  // cr[k]: contributions to node A ^ k
#pragma unroll
  for (int B = 0; B < 4; ++B) {
    const double NB = (B == 0) ? QA : QB;
    const double c = uq[0] * G.g[B][0] + uq[1] * G.g[B][1] + uq[2] * G.g[B][2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cr[B][i] = w * (NB * gal[i] + c * sv[i]);
      cr[B][4 + i] = w * NB * sv[i];
    }
    cr[B][3] = w * p.inv_rho * (G.g[B][0] * sv[0] + G.g[B][1] * sv[1] + G.g[B][2] * sv[2]);
  }
  quad_gather_rows(cr, res);
  const double V = G.V;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    res[i] += V * (p.mu * (gA[0] * Gm[i][0] + gA[1] * Gm[i][1] + gA[2] * Gm[i][2]) - gA[i] * pbar);
  res[3] += w * (Gm[0][0] + Gm[1][1] + Gm[2][2]);
  return base;
}

// Exact directional derivative of k_elem_residual along the direction
// samples Sv (dtau = -tau^3 u.xi du from eq. tau), plus shift * int N_A N_B
// on the velocity rows.
template <typename R>
__device__ __forceinline__ int64_t jvp_exact_lane(const DevMesh& m, const Phys& p,
                                                  const R* __restrict__ Sy,
                                                  const R* __restrict__ Sv, int64_t t, int s,
                                                  int A, R res[NCH]) {
  const int N = p.N;
  GeoT<R> G;  // G.g[k] = grad N_(A ^ k)
  load_geo_lane(m.geo, m.ne, t, A, G);
  const R* gA = G.g[0];
  const int64_t base = (int64_t)m.tets[A * m.ne + t] * NCH * N + s;
  const R* q = Sy + base;
  const R* d = Sv + base;
  R u[3], hu[3], du[3], dhu[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    u[i] = q[i * N];
    hu[i] = q[(4 + i) * N];
    du[i] = d[i * N];
    dhu[i] = d[(4 + i) * N];
  }
  const R pr = q[3 * N], dp = d[3 * N];
  R Gm[3][3], dG[3][3], gp[3], dgp[3], uq[3], hq[3], duq[3], dhq[3], dus[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Gm[i][j] = quad_sum(u[i] * gA[j]);
      dG[i][j] = quad_sum(du[i] * gA[j]);
    }
    gp[i] = quad_sum(pr * gA[i]);
    dgp[i] = quad_sum(dp * gA[i]);
    dus[i] = quad_sum(du[i]);
    uq[i] = R(QB) * quad_sum(u[i]) + R(QA - QB) * u[i];
    hq[i] = R(QB) * quad_sum(hu[i]) + R(QA - QB) * hu[i];
    duq[i] = R(QB) * dus[i] + R(QA - QB) * du[i];
    dhq[i] = R(QB) * quad_sum(dhu[i]) + R(QA - QB) * dhu[i];
  }
  const R dpbar = R(0.25) * quad_sum(dp);
  const R rho = (R)p.rho;
  const R w = R(0.25) * G.V;
  R adv[3], dadv[3], xu[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    adv[i] = uq[0] * Gm[i][0] + uq[1] * Gm[i][1] + uq[2] * Gm[i][2];
    dadv[i] = duq[0] * Gm[i][0] + duq[1] * Gm[i][1] + duq[2] * Gm[i][2]
            + uq[0] * dG[i][0] + uq[1] * dG[i][1] + uq[2] * dG[i][2];
  }
  xi_mul(G, uq, xu);
  const R tau =
      rsqrt_nr(uq[0] * xu[0] + uq[1] * xu[1] + uq[2] * xu[2] + R(p.C_I * p.nu * p.nu) * G.xixi +
               R(p.tau_add));
  const R dtau = -tau * tau * tau * (xu[0] * duq[0] + xu[1] * duq[1] + xu[2] * duq[2]);
  R sv[3], ds[3], dgal[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const R L = rho * (hq[i] + adv[i]) + gp[i];
    dgal[i] = rho * (dhq[i] + dadv[i]);
    sv[i] = tau * L;
    ds[i] = dtau * L + tau * (dgal[i] + dgp[i]);
  }
  R cr[4][NCH];  // cr[k]: contributions to node A ^ k
#pragma unroll
  for (int B = 0; B < 4; ++B) {
    const R NB = (B == 0) ? R(QA) : R(QB);
    const R c = uq[0] * G.g[B][0] + uq[1] * G.g[B][1] + uq[2] * G.g[B][2];
    const R dc = duq[0] * G.g[B][0] + duq[1] * G.g[B][1] + duq[2] * G.g[B][2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cr[B][i] = w * (NB * dgal[i] + dc * sv[i] + c * ds[i]);
      cr[B][4 + i] = w * NB * ds[i];
    }
    cr[B][3] = w * R(p.inv_rho) * (G.g[B][0] * ds[0] + G.g[B][1] * ds[1] + G.g[B][2] * ds[2]);
  }
  quad_gather_rows(cr, res);
  const R V = G.V;
  const R ms = R(p.shift) * V * R(1.0 / 20.0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
    res[i] += V * (R(p.mu) * (gA[0] * dG[i][0] + gA[1] * dG[i][1] + gA[2] * dG[i][2]) - gA[i] * dpbar)
            + ms * (dus[i] + du[i]);
  res[3] += w * (dG[0][0] + dG[1][1] + dG[2][2]);
  return base;
}

// Element block of EB consecutive tetrahedra per workgroup: the lanes loop
// over (element, sample, node) quads, add their node rows into an LDS
// accumulator indexed by the block's unique nodes (precomputed on the host),
// and the workgroup then adds each unique node's 7 x N block to the global
// accumulator once (contiguous atomics), instead of one atomic per element
// row.  Device-scope FP64 atomics are resolved beyond the per-XCD L2, so
// their count is what this removes.
template <int KIND, typename R>
__global__ void __launch_bounds__(BLK)
k_elem_block(DevMesh m, Phys p, const R* __restrict__ Sy, const R* __restrict__ Sv,
             R* __restrict__ acc, ElemBlocks eb, int64_t nlogical) {
  // [U][NCH][N], FP64 also in the FP32 kernel: 32-bit LDS atomics on this
  // access pattern stall on bank conflicts, 64-bit ones do not
  extern __shared__ double sacc[];
  const int64_t b = xcd_block(nlogical);
  if (b < 0) return;
  const int N = p.N;
  const int CN = NCH * N;
  const int64_t e0 = b * eb.size;
  const int nel = (int)min<int64_t>(eb.size, m.ne - e0);
  const int32_t p0 = eb.ptr[b];
  const int U = eb.ptr[b + 1] - p0;
  for (int i = threadIdx.x; i < U * CN; i += BLK) sacc[i] = 0.0;
  __syncthreads();
  // a replayed graph reads the pseudo-time shift from device memory, once
  // per workgroup, so that the lane code sees a plain value
  Phys q = p;
  if (KIND == 1 && p.shift_dev) q.shift = *p.shift_dev;
  const int total = nel * N * 4;
  for (int it = threadIdx.x; it < total; it += BLK) {  // quads stay aligned (BLK % 4 == 0)
    const int A = it & 3;
    const int ts = it >> 2;
    const int el = ts / N;
    const int s = ts - el * N;
    const int64_t t = e0 + el;
    R r[NCH];
    if constexpr (KIND == 0)
      residual_lane(m, q, Sy, t, s, A, r);
    else
      jvp_exact_lane<R>(m, q, Sy, Sv, t, s, A, r);
    double* dst = sacc + eb.slot[A * m.ne + t] * CN + s;
#pragma unroll
    for (int c = 0; c < NCH; ++c)
      __hip_atomic_fetch_add(dst + c * N, (double)r[c], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < U * CN; i += BLK) {
    const int u = i / CN;
    const int r = i - u * CN;
    atomic_add(acc + (int64_t)eb.nodes[p0 + u] * CN + r, (R)sacc[i]);
  }
}

// The paper's tangent C + P (eqs. K_mat, ctangent) applied matrix-free:
// advection and tau frozen at the state, stabilisation time terms dropped,
// Galerkin time term rho int N_A H du (the F block) kept; plus shift mass.
__global__ void __launch_bounds__(BLK)
k_elem_jvp_paper(DevMesh m, Phys p, const double* __restrict__ Sy, const double* __restrict__ Sv,
                 double* __restrict__ acc, int64_t nlogical) {
  const int64_t lb = xcd_block(nlogical);
  if (lb < 0) return;
  const int N = p.N;
  const int64_t gid = lb * BLK + threadIdx.x;
  if (gid >= m.ne * N) return;
  const int64_t t = gid / N;
  const int s = (int)(gid - t * N);
  Geo G;
  load_geo(m.geo, m.ne, t, G);
  int64_t base[4];
  double u[4][3], du[4][3], dhu[4][3], dp[4];
#pragma unroll
  for (int A = 0; A < 4; ++A) {
    const int64_t a = m.tets[A * m.ne + t];
    base[A] = a * NCH * N + s;
    const double* q = Sy + base[A];
    const double* d = Sv + base[A];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      u[A][i] = q[i * N];
      du[A][i] = d[i * N];
      dhu[A][i] = d[(4 + i) * N];
    }
    dp[A] = d[3 * N];
  }
  double dG[3][3], dgp[3], us[3], dus[3], dhs[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    dgp[i] = 0.0;
    us[i] = u[0][i] + u[1][i] + u[2][i] + u[3][i];
    dus[i] = du[0][i] + du[1][i] + du[2][i] + du[3][i];
    dhs[i] = dhu[0][i] + dhu[1][i] + dhu[2][i] + dhu[3][i];
#pragma unroll
    for (int j = 0; j < 3; ++j) dG[i][j] = 0.0;
  }
#pragma unroll
  for (int A = 0; A < 4; ++A)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      dgp[i] += dp[A] * G.g[A][i];
#pragma unroll
      for (int j = 0; j < 3; ++j) dG[i][j] += du[A][i] * G.g[A][j];
    }
  const double ddiv = dG[0][0] + dG[1][1] + dG[2][2];
  const double dpbar = 0.25 * (dp[0] + dp[1] + dp[2] + dp[3]);
  const double rho = p.rho;
  const double kap0 = p.C_I * p.nu * p.nu * G.xixi + p.tau_add;
  const double w = 0.25 * G.V;
  double rm[4][3], rc[4], z[4][3], dS[3] = {0, 0, 0};
#pragma unroll
  for (int A = 0; A < 4; ++A) {
    rc[A] = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) rm[A][i] = z[A][i] = 0.0;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double uq[3], dhq[3], dadv[3], xu[3], ds[3], c[4];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      uq[i] = QB * us[i] + (QA - QB) * u[q][i];
      dhq[i] = QB * dhs[i] + (QA - QB) * dhu[q][i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) dadv[i] = uq[0] * dG[i][0] + uq[1] * dG[i][1] + uq[2] * dG[i][2];
    xi_mul(G, uq, xu);
    const double tau = 1.0 / sqrt(uq[0] * xu[0] + uq[1] * xu[1] + uq[2] * xu[2] + kap0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ds[i] = tau * (rho * dadv[i] + dgp[i]);
      dS[i] += w * ds[i];
    }
#pragma unroll
    for (int A = 0; A < 4; ++A) c[A] = uq[0] * G.g[A][0] + uq[1] * G.g[A][1] + uq[2] * G.g[A][2];
#pragma unroll
    for (int A = 0; A < 4; ++A) {
      const double NA = (A == q) ? QA : QB;
#pragma unroll
      for (int i = 0; i < 3; ++i) rm[A][i] += w * (NA * rho * (dhq[i] + dadv[i]) + c[A] * ds[i]);
    }
  }
  const double V = G.V;
  const double ms = p.shift * V * (1.0 / 20.0);
#pragma unroll
  for (int A = 0; A < 4; ++A) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
      rm[A][i] += V * (p.mu * (G.g[A][0] * dG[i][0] + G.g[A][1] * dG[i][1] + G.g[A][2] * dG[i][2])
                       - G.g[A][i] * dpbar)
                + ms * (dus[i] + du[A][i]);
    rc[A] = w * ddiv + (G.g[A][0] * dS[0] + G.g[A][1] * dS[1] + G.g[A][2] * dS[2]) / rho;
  }
  scatter_rows(acc, base, N, rm, rc, z, false);
}

// Diagonal of P (Section 2.3: the Jacobi preconditioner): K_AA and L_AA per
// sample, plus shift * int N_A^2 = shift V/10.  dg[a][0|1][s].  With
// time_terms, also the nodal integrals that the exact Jacobian's
// stabilisation time terms multiply: T_AA = int tau N_A^2 in dg[a][2][s]
// and X_AA = int rho tau (u.grad N_A) N_A in dg[a][3][s] (dg has 4 channels).
__global__ void __launch_bounds__(BLK)
k_elem_jacobi(DevMesh m, Phys p, const double* __restrict__ Sy, double* __restrict__ dg,
              int time_terms, int64_t nlogical) {
  const int64_t lb = xcd_block(nlogical);
  if (lb < 0) return;
  const int N = p.N;
  const int64_t gid = lb * BLK + threadIdx.x;
  if (gid >= m.ne * N) return;
  const int64_t t = gid / N;
  const int s = (int)(gid - t * N);
  Geo G;
  load_geo(m.geo, m.ne, t, G);
  int64_t node[4];
  double u[4][3];
#pragma unroll
  for (int A = 0; A < 4; ++A) {
    node[A] = m.tets[A * m.ne + t];
    const double* q = Sy + node[A] * NCH * N + s;
#pragma unroll
    for (int i = 0; i < 3; ++i) u[A][i] = q[i * N];
  }
  double us[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) us[i] = u[0][i] + u[1][i] + u[2][i] + u[3][i];
  const double rho = p.rho;
  const double kap0 = p.C_I * p.nu * p.nu * G.xixi + p.tau_add;
  const double w = 0.25 * G.V;
  double kd[4] = {0, 0, 0, 0}, ld[4] = {0, 0, 0, 0}, td[4] = {0, 0, 0, 0}, xd[4] = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double uq[3], xu[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) uq[i] = QB * us[i] + (QA - QB) * u[q][i];
    xi_mul(G, uq, xu);
    const double tau = 1.0 / sqrt(uq[0] * xu[0] + uq[1] * xu[1] + uq[2] * xu[2] + kap0);
#pragma unroll
    for (int A = 0; A < 4; ++A) {
      const double NA = (A == q) ? QA : QB;
      const double c = uq[0] * G.g[A][0] + uq[1] * G.g[A][1] + uq[2] * G.g[A][2];
      kd[A] += w * (rho * NA * c + rho * tau * c * c);
      ld[A] += w * tau;
      td[A] += w * tau * NA * NA;
      xd[A] += w * rho * tau * c * NA;
    }
  }
  const int nc = time_terms ? 4 : 2;
#pragma unroll
  for (int A = 0; A < 4; ++A) {
    const double gg = G.g[A][0] * G.g[A][0] + G.g[A][1] * G.g[A][1] + G.g[A][2] * G.g[A][2];
    double* d = dg + (node[A] * nc) * N + s;
    atomic_add(d, kd[A] + p.mu * G.V * gg + p.shift * G.V * 0.1);
    atomic_add(d + N, ld[A] * gg / rho);
    if (time_terms) {
      atomic_add(d + 2 * N, td[A]);
      atomic_add(d + 3 * N, xd[A]);
    }
  }
}

// --------------------------------------------------------------- faces

// Q[k][s] = sum over outlet k's faces of area * (mean nodal u) . n; one
// workgroup per sample, per-outlet partial sums in LDS.
template <typename R>
__global__ void __launch_bounds__(BLK)
k_outlet_flux(DevMesh m, int N, const R* __restrict__ S, double* __restrict__ Q, int64_t chunk) {
  __shared__ double sq[64];
  const int s = blockIdx.x;
  const int64_t f0 = (int64_t)blockIdx.y * chunk;
  const int64_t f1 = min<int64_t>(m.nof, f0 + chunk);
  for (int k = threadIdx.x; k < m.n_out; k += BLK) sq[k] = 0.0;
  __syncthreads();
  for (int64_t f = f0 + threadIdx.x; f < f1; f += BLK) {
    double ub[3] = {0, 0, 0};
#pragma unroll
    for (int A = 0; A < 3; ++A) {
      const R* q = S + (int64_t)m.of[A * m.nof + f] * NCH * N + s;
      ub[0] += q[0];
      ub[1] += q[N];
      ub[2] += q[2 * N];
    }
    const double v = m.ofn[3 * m.nof + f] / 3.0
                   * (ub[0] * m.ofn[f] + ub[1] * m.ofn[m.nof + f] + ub[2] * m.ofn[2 * m.nof + f]);
    atomicAdd(&sq[m.oid[f]], v);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < m.n_out; k += BLK) atomicAdd(&Q[k * N + s], sq[k]);
}

// Outlet rows: -int N_A h n_i with h = hs - R Q, and the backflow term
// -int N_A (rho beta/2) min(u.n, 0) u_i on the 3-point rule (Section 2.3).
__global__ void __launch_bounds__(BLK)
k_face_residual(DevMesh m, Phys p, const double* __restrict__ S, const double* __restrict__ hs,
                const double* __restrict__ Rk, const double* __restrict__ Q,
                double* __restrict__ acc) {
  const int N = p.N;
  const int64_t gid = (int64_t)blockIdx.x * BLK + threadIdx.x;
  if (gid >= m.nof * N) return;
  const int64_t f = gid / N;
  const int s = (int)(gid - f * N);
  const double nx = m.ofn[f], ny = m.ofn[m.nof + f], nz = m.ofn[2 * m.nof + f];
  const double area = m.ofn[3 * m.nof + f];
  const int k = m.oid[f];
  double h = hs ? hs[k * N + s] : 0.0;
  if (Rk) h -= Rk[k] * Q[k * N + s];
  int64_t base[3];
  double u[3][3], r[3][3];
#pragma unroll
  for (int A = 0; A < 3; ++A) {
    base[A] = (int64_t)m.of[A * m.nof + f] * NCH * N + s;
#pragma unroll
    for (int i = 0; i < 3; ++i) u[A][i] = S[base[A] + i * N];
    const double hn = -h * area / 3.0;
    r[A][0] = hn * nx;
    r[A][1] = hn * ny;
    r[A][2] = hn * nz;
  }
  if (p.backflow) {
    const double coef = -(area / 3.0) * 0.5 * p.rho * p.beta;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double uq[3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
        uq[i] = TRI_B * (u[0][i] + u[1][i] + u[2][i]) + (TRI_A - TRI_B) * u[q][i];
      const double un = uq[0] * nx + uq[1] * ny + uq[2] * nz;
      if (un < 0.0) {
#pragma unroll
        for (int A = 0; A < 3; ++A) {
          const double NA = (A == q) ? TRI_A : TRI_B;
#pragma unroll
          for (int i = 0; i < 3; ++i) r[A][i] += coef * un * NA * uq[i];
        }
      }
    }
  }
#pragma unroll
  for (int A = 0; A < 3; ++A)
#pragma unroll
    for (int i = 0; i < 3; ++i) atomic_add(acc + base[A] + i * N, r[A][i]);
}

// Directional derivative of k_face_residual: -int N_A (-R dQ) n_i and the
// backflow tangent with the kink's derivative taken as zero at u.n = 0.
template <typename R>
__global__ void __launch_bounds__(BLK)
k_face_jvp(DevMesh m, Phys p, const R* __restrict__ Sy, const R* __restrict__ Sv,
           const double* __restrict__ Rk, const double* __restrict__ dQ, R* __restrict__ acc) {
  const int N = p.N;
  const int64_t gid = (int64_t)blockIdx.x * BLK + threadIdx.x;
  if (gid >= m.nof * N) return;
  const int64_t f = gid / N;
  const int s = (int)(gid - f * N);
  const double nx = m.ofn[f], ny = m.ofn[m.nof + f], nz = m.ofn[2 * m.nof + f];
  const double area = m.ofn[3 * m.nof + f];
  const int k = m.oid[f];
  const double dh = Rk ? -Rk[k] * dQ[k * N + s] : 0.0;
  int64_t base[3];
  double u[3][3], du[3][3], r[3][3];
#pragma unroll
  for (int A = 0; A < 3; ++A) {
    base[A] = (int64_t)m.of[A * m.nof + f] * NCH * N + s;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      u[A][i] = Sy[base[A] + i * N];
      du[A][i] = Sv[base[A] + i * N];
    }
    const double hn = -dh * area / 3.0;
    r[A][0] = hn * nx;
    r[A][1] = hn * ny;
    r[A][2] = hn * nz;
  }
  if (p.backflow) {
    const double coef = -(area / 3.0) * 0.5 * p.rho * p.beta;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double uq[3], duq[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        uq[i] = TRI_B * (u[0][i] + u[1][i] + u[2][i]) + (TRI_A - TRI_B) * u[q][i];
        duq[i] = TRI_B * (du[0][i] + du[1][i] + du[2][i]) + (TRI_A - TRI_B) * du[q][i];
      }
      const double un = uq[0] * nx + uq[1] * ny + uq[2] * nz;
      if (un < 0.0) {
        const double dun = duq[0] * nx + duq[1] * ny + duq[2] * nz;
#pragma unroll
        for (int A = 0; A < 3; ++A) {
          const double NA = (A == q) ? TRI_A : TRI_B;
#pragma unroll
          for (int i = 0; i < 3; ++i) r[A][i] += coef * NA * (dun * uq[i] + un * duq[i]);
        }
      }
    }
  }
#pragma unroll
  for (int A = 0; A < 3; ++A)
#pragma unroll
    for (int i = 0; i < 3; ++i) atomic_add(acc + base[A] + i * N, (R)r[A][i]);
}

// dg[a][c][s] -> D[c][s][a] (field-major), Dirichlet velocity rows = 1;
// optionally dinv[a][c][s] = 1 / diag.
__global__ void __launch_bounds__(BLK)
k_jacobi_out(int64_t n, int N, int nc, const uint8_t* __restrict__ dmask, double* __restrict__ dg,
             double* __restrict__ D, double* __restrict__ dinv) {
  const int64_t gid = (int64_t)blockIdx.x * BLK + threadIdx.x;
  if (gid >= n * 2 * N) return;
  const int64_t a = gid / (2 * N);
  const int r = (int)(gid - a * 2 * N);
  const int c = r / N;
  const int s = r - c * N;
  double* d = dg + (a * nc + c) * N + s;
  double v = *d;
  if (c == 0 && dmask[a]) v = 1.0;
  *d = v;
  if (D) D[((int64_t)c * N + s) * n + a] = v;
  if (dinv) dinv[gid] = 1.0 / v;
}

// -------------------------------------------------------------- vectors

template <int G, typename T>
__global__ void __launch_bounds__(BLK)
k_dots(const T* __restrict__ Q, int64_t ld, int k0, int kc, const T* __restrict__ w,
       int64_t L, double* __restrict__ partial, int nblk) {
  __shared__ double red[G][BLK / 64];
  double acc[G];
#pragma unroll
  for (int j = 0; j < G; ++j) acc[j] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < L; i += stride) {
    const double wi = (double)w[i];
#pragma unroll
    for (int j = 0; j < G; ++j)
      if (j < kc) acc[j] += (double)Q[(int64_t)(k0 + j) * ld + i] * wi;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < G; ++j) {
    double v = acc[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) red[j][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < G && threadIdx.x < kc) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < BLK / 64; ++q) v += red[threadIdx.x][q];
    partial[(int64_t)(k0 + threadIdx.x) * nblk + blockIdx.x] = v;
  }
}

__global__ void __launch_bounds__(BLK)
k_reduce_rows(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
  __shared__ double red[BLK / 64];
  const int j = blockIdx.x;
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += BLK) v += partial[(int64_t)j * nblk + i];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if (lane == 0) red[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < BLK / 64; ++q) t += red[q];
    out[j] = t;
  }
}

// Block sum of v into red (BLK / 64 slots); result valid in thread 0.
__device__ inline double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < BLK / 64; ++q) t += red[q];
  return t;
}

// Per-workgroup partial dot products Q_j . w for all j < k in one launch:
// blockIdx.y selects a group of G basis vectors, blockIdx.x a slice of the
// vectors; partial[j][blockIdx.x] (k_reduce_rows finishes the sums).
template <int G, typename T>
__global__ void __launch_bounds__(BLK)
k_mdots(const T* __restrict__ Q, int64_t ld, int k, const T* __restrict__ w, int64_t L,
        double* __restrict__ partial) {
  __shared__ double red[BLK / 64];
  const int k0 = blockIdx.y * G;
  const int kc = min(G, k - k0);
  const int nb = gridDim.x;
  double acc[G];
#pragma unroll
  for (int j = 0; j < G; ++j) acc[j] = 0.0;
  const int64_t stride = (int64_t)nb * BLK;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < L; i += stride) {
    const double wi = (double)w[i];
#pragma unroll
    for (int j = 0; j < G; ++j)
      if (j < kc) acc[j] += (double)Q[(int64_t)(k0 + j) * ld + i] * wi;
  }
#pragma unroll
  for (int j = 0; j < G; ++j) {
    const double t = block_sum(acc[j], red);
    if (threadIdx.x == 0 && j < kc) partial[(int64_t)(k0 + j) * nb + blockIdx.x] = t;
  }
}

// 16-byte packs of Krylov vector entries (4 FP32 or 2 FP64 values): one
// load or store instruction moves a full 16 bytes per lane.
template <typename T>
struct alignas(16) Pack16 {
  static constexpr int W = 16 / sizeof(T);
  T v[W];
};

// k_mdots on 16-byte packs (L and ld multiples of the pack width, vectors
// 16-byte aligned).
template <int G, typename T>
__global__ void __launch_bounds__(BLK)
k_mdots_v(const T* __restrict__ Q, int64_t ld, int k, const T* __restrict__ w, int64_t L,
          double* __restrict__ partial) {
  using P = Pack16<T>;
  __shared__ double red[BLK / 64];
  const int k0 = blockIdx.y * G;
  const int kc = min(G, k - k0);
  const int nb = gridDim.x;
  const int64_t nc = L / P::W, ldc = ld / P::W;
  const P* Qp = reinterpret_cast<const P*>(Q);
  const P* wp = reinterpret_cast<const P*>(w);
  double acc[G];
#pragma unroll
  for (int j = 0; j < G; ++j) acc[j] = 0.0;
  const int64_t stride = (int64_t)nb * BLK;
  for (int64_t c = (int64_t)blockIdx.x * BLK + threadIdx.x; c < nc; c += stride) {
    const P wc = wp[c];
#pragma unroll
    for (int j = 0; j < G; ++j)
      if (j < kc) {
        const P q = Qp[(int64_t)(k0 + j) * ldc + c];
#pragma unroll
        for (int e = 0; e < P::W; ++e) acc[j] += (double)q.v[e] * (double)wc.v[e];
      }
  }
#pragma unroll
  for (int j = 0; j < G; ++j) {
    const double t = block_sum(acc[j], red);
    if (threadIdx.x == 0 && j < kc) partial[(int64_t)(k0 + j) * nb + blockIdx.x] = t;
  }
}

// k_axpy_norm on 16-byte packs.
template <typename T>
__global__ void __launch_bounds__(BLK)
k_axpy_norm_v(T* __restrict__ w, const T* __restrict__ Q, int64_t ld, int k,
              const double* __restrict__ h, int64_t L, double* __restrict__ partial) {
  using P = Pack16<T>;
  __shared__ double red[BLK / 64];
  const int64_t nc = L / P::W, ldc = ld / P::W;
  const P* Qp = reinterpret_cast<const P*>(Q);
  P* wp = reinterpret_cast<P*>(w);
  double s2 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t c = (int64_t)blockIdx.x * BLK + threadIdx.x; c < nc; c += stride) {
    double v[P::W];
#pragma unroll
    for (int e = 0; e < P::W; ++e) v[e] = 0.0;
    for (int j = 0; j < k; ++j) {
      const P q = Qp[(int64_t)j * ldc + c];
      const double hj = h[j];
#pragma unroll
      for (int e = 0; e < P::W; ++e) v[e] += hj * (double)q.v[e];
    }
    P wc = wp[c];
#pragma unroll
    for (int e = 0; e < P::W; ++e) {
      wc.v[e] = (T)((double)wc.v[e] - v[e]);
      s2 += (double)wc.v[e] * (double)wc.v[e];
    }
    wp[c] = wc;
  }
  const double t = block_sum(s2, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// k_axpy_multi on 16-byte packs.
template <typename T>
__global__ void __launch_bounds__(BLK)
k_axpy_multi_v(T* __restrict__ w, const T* __restrict__ Q, int64_t ld, int k,
               const double* __restrict__ h, double sign, int64_t L) {
  using P = Pack16<T>;
  const int64_t nc = L / P::W, ldc = ld / P::W;
  const P* Qp = reinterpret_cast<const P*>(Q);
  P* wp = reinterpret_cast<P*>(w);
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t c = (int64_t)blockIdx.x * BLK + threadIdx.x; c < nc; c += stride) {
    double v[P::W];
#pragma unroll
    for (int e = 0; e < P::W; ++e) v[e] = 0.0;
    for (int j = 0; j < k; ++j) {
      const P q = Qp[(int64_t)j * ldc + c];
      const double hj = h[j];
#pragma unroll
      for (int e = 0; e < P::W; ++e) v[e] += hj * (double)q.v[e];
    }
    P wc = wp[c];
#pragma unroll
    for (int e = 0; e < P::W; ++e) wc.v[e] = (T)((double)wc.v[e] + sign * v[e]);
    wp[c] = wc;
  }
}

// w -= sum_j h_j Q_j, with per-workgroup partials of |w|^2 of the result in
// partial[blockIdx.x] (k_reduce_rows finishes the sum).
template <typename T>
__global__ void __launch_bounds__(BLK)
k_axpy_norm(T* __restrict__ w, const T* __restrict__ Q, int64_t ld, int k,
            const double* __restrict__ h, int64_t L, double* __restrict__ partial) {
  __shared__ double red[BLK / 64];
  double s2 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < L; i += stride) {
    double v = 0.0;
    for (int j = 0; j < k; ++j) v += h[j] * (double)Q[(int64_t)j * ld + i];
    const T wn = (T)((double)w[i] - v);
    w[i] = wn;
    s2 += (double)wn * (double)wn;
  }
  const double t = block_sum(s2, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

template <typename T>
__global__ void __launch_bounds__(BLK)
k_axpy_multi(T* __restrict__ w, const T* __restrict__ Q, int64_t ld, int k,
             const double* __restrict__ h, double sign, int64_t L) {
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < L; i += stride) {
    double v = 0.0;
    for (int j = 0; j < k; ++j) v += h[j] * (double)Q[(int64_t)j * ld + i];
    w[i] = (T)((double)w[i] + sign * v);
  }
}

template <typename T>
__global__ void __launch_bounds__(BLK)
k_scale(T* __restrict__ x, int64_t L, double s) {
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < L; i += stride)
    x[i] = (T)((double)x[i] * s);
}

// x /= sqrt(*nrm2) when that norm is positive and finite (Arnoldi
// normalisation without a round trip to the host).
template <typename T>
__global__ void __launch_bounds__(BLK)
k_scale_inv_norm(T* __restrict__ x, int64_t L, const double* __restrict__ nrm2) {
  const double nv = sqrt(fmax(*nrm2, 0.0));
  if (!(nv > 0.0) || !isfinite(nv)) return;
  const double s = 1.0 / nv;
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < L; i += stride)
    x[i] = (T)((double)x[i] * s);
}

// out[s] = mean over the listed inlet nodes of |u(t_s)|, u(t_s) from the
// modal Dirichlet data d[3][N][n] (the characteristic speed of the CFL rule).
__global__ void __launch_bounds__(BLK)
k_inlet_speed(const double* __restrict__ d, int64_t n, int N, const int32_t* __restrict__ nodes,
              int64_t ni, const double* __restrict__ tab, double* __restrict__ out) {
  __shared__ double red[BLK / 64];
  const int s = blockIdx.x;
  const double* Binv = tab + (size_t)TAB_BINV * N * N + (size_t)s * N;
  double sum = 0.0;
  for (int64_t k = threadIdx.x; k < ni; k += BLK) {
    const int64_t a = nodes[k];
    double g2 = 0.0;
    for (int i = 0; i < 3; ++i) {
      double v = 0.0;
      for (int mm = 0; mm < N; ++mm) v += Binv[mm] * d[((int64_t)i * N + mm) * n + a];
      g2 += v * v;
    }
    sum += sqrt(g2);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_down(sum, o, 64);
  if (lane == 0) red[wv] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < BLK / 64; ++q) t += red[q];
    out[s] = t / (double)ni;
  }
}

template <typename T>
__global__ void __launch_bounds__(BLK)
k_fill(T* __restrict__ x, int64_t L, double v) {
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < L; i += stride) x[i] = (T)v;
}

template <typename TD, typename TS>
__global__ void __launch_bounds__(BLK)
k_copy_scaled(TD* __restrict__ d, const TS* __restrict__ x, int64_t L, double s) {
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < L; i += stride)
    d[i] = (TD)(s * (double)x[i]);
}

// out[s] += sum over nodes of X[a][ch][s] (X has nch channels of N samples);
// one workgroup per (sample, chunk of nodes)
__global__ void __launch_bounds__(BLK)
k_channel_sum(const double* __restrict__ X, int64_t n, int nch, int N, int ch, int64_t chunk,
              double* __restrict__ out) {
  __shared__ double red[BLK];
  const int s = blockIdx.x;
  const int64_t a0 = (int64_t)blockIdx.y * chunk;
  const int64_t a1 = min<int64_t>(n, a0 + chunk);
  double v = 0.0;
  for (int64_t a = a0 + threadIdx.x; a < a1; a += BLK) v += X[(a * nch + ch) * N + s];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int off = BLK / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(&out[s], red[0]);
}

// y = a + alpha (b - a) (damped Newton step between two states)
__global__ void __launch_bounds__(BLK)
k_blend(double* __restrict__ y, const double* __restrict__ a, const double* __restrict__ b,
        int64_t L, double alpha) {
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < L; i += stride)
    y[i] = a[i] + alpha * (b[i] - a[i]);
}

// y[a][c][s] += s * dinv[a][c<3?0:1][s] * u[a][c][s] for c < 4, skipping the
// velocity entries of Dirichlet nodes.  y has nch_y channels per node.
template <typename TU>
__global__ void __launch_bounds__(BLK)
k_mul_dinv_add(double* __restrict__ y, const TU* __restrict__ u,
               const double* __restrict__ dinv, const uint8_t* __restrict__ dmask, int64_t n,
               int N, int nch_y, int nch_u, double s) {
  const int64_t gid = (int64_t)blockIdx.x * BLK + threadIdx.x;
  if (gid >= n * 4 * N) return;
  const int64_t a = gid / (4 * N);
  const int r = (int)(gid - a * 4 * N);
  const int c = r / N;
  const int sm = r - c * N;
  if (c < 3 && dmask[a]) return;
  const double d = dinv ? dinv[(a * 2 + (c < 3 ? 0 : 1)) * N + sm] : 1.0;
  y[(a * nch_y + c) * N + sm] += s * d * (double)u[(a * nch_u + c) * N + sm];
}

__global__ void __launch_bounds__(BLK)
k_nonfinite(const double* __restrict__ x, int64_t L, int* __restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * BLK;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < L; i += stride)
    bad |= !isfinite(x[i]);
  if (bad) atomicOr(flag, 1);
}

inline unsigned tiles(int64_t n) { return (unsigned)((n + TN - 1) / TN); }
inline unsigned blocks_for(int64_t work) { return (unsigned)((work + BLK - 1) / BLK); }
inline unsigned stream_blocks(int64_t L) {
  int64_t b = (L + BLK - 1) / BLK;
  return (unsigned)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

}  // namespace

// ------------------------------------------------------------- launchers

// Dynamic LDS of one workgroup allowed on the current device (cached per
// device); launchers refuse larger requests instead of launching them.
size_t lds_limit() {
  static std::atomic<int64_t> cache[64];
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= 64) return 65536;
  int64_t v = cache[d].load(std::memory_order_relaxed);
  if (v == 0) {
    int a = 0;
    if (hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, d) != hipSuccess ||
        a <= 0)
      a = 65536;
    v = a;
    cache[d].store(v, std::memory_order_relaxed);
  }
  return (size_t)v;
}

template <typename TI, typename TO, int TL>
hipError_t modal_to_samples_tl(const DevMesh& m, int N, const TI* Y, const double* dir,
                               int zero_dirichlet, const double* tab, TO* S, TO* acc_zero,
                               double* q_zero, int nq, hipStream_t st) {
  const size_t lds = sizeof(double) * (4 * N * TL + 2 * N * N);
  if (lds > lds_limit()) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_modal_to_samples<TI, TO, TL>), dim3((unsigned)((m.n + TL - 1) / TL)),
                     dim3(BLK), lds, st, m.n, N, Y, dir, m.dmask, zero_dirichlet, tab, S, acc_zero,
                     q_zero, nq);
  return hipGetLastError();
}

template <typename TA, typename TO, int TL>
hipError_t samples_to_modal_tl(const DevMesh& m, int N, const TA* acc, int use_z,
                               int zero_dir_rows, int in_ch, const double* tab, TO* R,
                               hipStream_t st) {
  const size_t lds = sizeof(double) * (TL * in_ch * N + 2 * N * N);
  if (lds > lds_limit()) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_samples_to_modal<TA, TO, TL>), dim3((unsigned)((m.n + TL - 1) / TL)),
                     dim3(BLK), lds, st, m.n, N, acc, use_z, zero_dir_rows, in_ch, m.dmask, tab,
                     R);
  return hipGetLastError();
}

template <typename TI, typename TO>
hipError_t modal_to_samples(const DevMesh& m, int N, const TI* Y, const double* dir,
                            int zero_dirichlet, const double* tab, TO* S, TO* acc_zero,
                            double* q_zero, int nq, hipStream_t st) {
  if (m.n == 0) return hipSuccess;
  // FP64 output: 16-node tiles (more workgroups per CU in flight); FP32
  // output: 32-node tiles for the 32 x 32 MFMA path (N <= 32), else 16
  if (std::is_same<TO, float>::value && N <= 32)
    return modal_to_samples_tl<TI, TO, TN>(m, N, Y, dir, zero_dirichlet, tab, S, acc_zero, q_zero,
                                           nq, st);
  return modal_to_samples_tl<TI, TO, 16>(m, N, Y, dir, zero_dirichlet, tab, S, acc_zero, q_zero,
                                         nq, st);
}

template <typename TA, typename TO>
hipError_t samples_to_modal(const DevMesh& m, int N, const TA* acc, int use_z, int zero_dir_rows,
                            int in_ch, const double* tab, TO* R, hipStream_t st) {
  if (m.n == 0) return hipSuccess;
  // FP64 output: 16-node tiles (half the LDS, twice the workgroups per CU in
  // flight); FP32 output: 32-node tiles for the 32 x 32 MFMA path (N <= 32)
  if (std::is_same<TO, float>::value && N <= 32)
    return samples_to_modal_tl<TA, TO, TN>(m, N, acc, use_z, zero_dir_rows, in_ch, tab, R, st);
  return samples_to_modal_tl<TA, TO, 16>(m, N, acc, use_z, zero_dir_rows, in_ch, tab, R, st);
}

template <typename TQ, typename TS>
hipError_t prepare_direction(const DevMesh& m, int N, const TQ* q, int in_ch, const double* dinv,
                             const double* binv, int zero_dirichlet, const double* tab, TS* Sv,
                             TS* acc_zero, double* q_zero, int nq, hipStream_t st) {
  const size_t lds = sizeof(double) * (TN * 4 * N + N * N + (binv ? TN * 3 * N : 0));
  if (lds > lds_limit()) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_prepare<TQ, TS>), dim3(tiles(m.n)), dim3(BLK), lds, st, m.n, N, q, in_ch,
                     dinv, binv, zero_dirichlet, m.dmask, tab, Sv, acc_zero, q_zero, nq);
  return hipGetLastError();
}

hipError_t block_factor(const DevMesh& m, int N, const double* dg, const double* mass,
                        double rho, const double* tab, double* binv, hipStream_t st) {
  if (N < 1 || N > 64) return hipErrorInvalidValue;
  const int P = 64 / N;
  const size_t lds = sizeof(double) * ((size_t)N * N * (1 + P) + (size_t)P * 4 * N);
  if (lds > lds_limit()) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)((m.n + P - 1) / P);
  hipLaunchKernelGGL(k_block_factor, dim3(grid), dim3(64), lds, st, m.n, N, P, dg, mass, rho, tab,
                     m.dmask, binv);
  return hipGetLastError();
}

template <typename TA, typename TO>
hipError_t finish_rows(const DevMesh& m, int N, const TA* acc, int use_z, const double* tab,
                       const TO* id_rows, TO* out, hipStream_t st) {
  const size_t lds = sizeof(double) * (TN * NCH * N + N * N);
  if (lds > lds_limit()) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_finish<TA, TO>), dim3(tiles(m.n)), dim3(BLK), lds, st, m.n, N, acc, use_z,
                     m.dmask, tab, id_rows, out);
  return hipGetLastError();
}

template <typename R>
hipError_t outlet_flux(const DevMesh& m, int N, const R* S, double* Q, hipStream_t st) {
  if (m.nof == 0) return hipSuccess;
  // Q must be zero on entry (the transform that fills S zeroes it): each
  // workgroup adds the flux of one chunk of outlet faces at one sample
  constexpr int64_t kChunk = 2048;
  const int64_t nch = (m.nof + kChunk - 1) / kChunk;
  hipLaunchKernelGGL((k_outlet_flux<R>), dim3(N, (unsigned)nch), dim3(BLK), 0, st, m, N, S, Q,
                     kChunk);
  return hipGetLastError();
}

hipError_t elem_residual(const DevMesh& m, const Phys& p, const double* S, double* acc,
                         const ElemBlocks& eb, hipStream_t st) {
  const int64_t nb = (m.ne + eb.size - 1) / eb.size;
  const size_t lds = sizeof(double) * (size_t)eb.max_unique * NCH * p.N;
  if (lds > lds_limit()) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_elem_block<0, double>), dim3(xcd_grid(nb)), dim3(BLK), lds, st, m, p, S, S,
                     acc, eb, nb);
  return hipGetLastError();
}

template <typename R>
hipError_t elem_jvp_exact(const DevMesh& m, const Phys& p, const R* Sy, const R* Sv, R* acc,
                          const ElemBlocks& eb, hipStream_t st) {
  const int64_t nb = (m.ne + eb.size - 1) / eb.size;
  const size_t lds = sizeof(double) * (size_t)eb.max_unique * NCH * p.N;
  if (lds > lds_limit()) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_elem_block<1, R>), dim3(xcd_grid(nb)), dim3(BLK), lds, st, m, p, Sy, Sv,
                     acc, eb, nb);
  return hipGetLastError();
}

hipError_t elem_jvp_paper(const DevMesh& m, const Phys& p, const double* Sy, const double* Sv,
                          double* acc, hipStream_t st) {
  const int64_t nb = (m.ne * p.N + BLK - 1) / BLK;
  hipLaunchKernelGGL(k_elem_jvp_paper, dim3(xcd_grid(nb)), dim3(BLK), 0, st, m, p, Sy, Sv, acc,
                     nb);
  return hipGetLastError();
}

hipError_t elem_jacobi(const DevMesh& m, const Phys& p, const double* Sy, double* dg,
                       int time_terms, hipStream_t st) {
  const int64_t nb = (m.ne * p.N + BLK - 1) / BLK;
  hipLaunchKernelGGL(k_elem_jacobi, dim3(xcd_grid(nb)), dim3(BLK), 0, st, m, p, Sy, dg,
                     time_terms, nb);
  return hipGetLastError();
}

hipError_t face_residual(const DevMesh& m, const Phys& p, const double* S, const double* hs,
                         const double* Rk, const double* Q, double* acc, hipStream_t st) {
  if (m.nof == 0) return hipSuccess;
  hipLaunchKernelGGL(k_face_residual, dim3(blocks_for(m.nof * p.N)), dim3(BLK), 0, st, m, p, S,
                     hs, Rk, Q, acc);
  return hipGetLastError();
}

template <typename R>
hipError_t face_jvp(const DevMesh& m, const Phys& p, const R* Sy, const R* Sv, const double* Rk,
                    const double* dQ, R* acc, hipStream_t st) {
  if (m.nof == 0) return hipSuccess;
  hipLaunchKernelGGL((k_face_jvp<R>), dim3(blocks_for(m.nof * p.N)), dim3(BLK), 0, st, m, p, Sy,
                     Sv, Rk, dQ, acc);
  return hipGetLastError();
}

hipError_t jacobi_out(const DevMesh& m, int N, int nc, const double* dg, double* D, double* dinv,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_out, dim3(blocks_for(m.n * 2 * N)), dim3(BLK), 0, st, m.n, N, nc,
                     m.dmask, const_cast<double*>(dg), D, dinv);
  return hipGetLastError();
}

template <typename T>
hipError_t vec_dots(const T* Q, int64_t ld, int k, const T* w, int64_t L, double* partial,
                    int nblk, double* out, hipStream_t st) {
  for (int k0 = 0; k0 < k; k0 += 8) {
    const int kc = k - k0 < 8 ? k - k0 : 8;
    hipLaunchKernelGGL((k_dots<8, T>), dim3(nblk), dim3(BLK), 0, st, Q, ld, k0, kc, w, L, partial,
                       nblk);
  }
  hipLaunchKernelGGL(k_reduce_rows, dim3(k), dim3(BLK), 0, st, partial, nblk, out);
  return hipGetLastError();
}

// The 16-byte pack kernels apply: whole packs, aligned rows.
template <typename T>
bool packable(int64_t L, int64_t ld, const T* Q, const T* w) {
  constexpr int W = Pack16<T>::W;
  return L % W == 0 && ld % W == 0 && ((uintptr_t)Q & 15) == 0 && ((uintptr_t)w & 15) == 0;
}

// workgroups per vector slice for the fused reductions: >= 4 elements per
// lane, at most nblk
inline unsigned red_blocks(int64_t L, int nblk) {
  const int64_t b = (L + 4 * BLK - 1) / (4 * BLK);
  return (unsigned)(b < 1 ? 1 : (b > nblk ? nblk : b));
}

template <typename T>
hipError_t vec_mdots(const T* Q, int64_t ld, int k, const T* w, int64_t L, double* partial,
                     int nblk, double* out, hipStream_t st) {
  const unsigned nb = red_blocks(L, nblk);
  const unsigned groups = (unsigned)((k + 7) / 8);
  if (packable<T>(L, ld, Q, w))
    hipLaunchKernelGGL((k_mdots_v<8, T>), dim3(nb, groups), dim3(BLK), 0, st, Q, ld, k, w, L,
                       partial);
  else
    hipLaunchKernelGGL((k_mdots<8, T>), dim3(nb, groups), dim3(BLK), 0, st, Q, ld, k, w, L,
                       partial);
  hipLaunchKernelGGL(k_reduce_rows, dim3(k), dim3(BLK), 0, st, partial, (int)nb, out);
  return hipGetLastError();
}

template <typename T>
hipError_t vec_axpy_norm(T* w, const T* Q, int64_t ld, int k, const double* h, int64_t L,
                         double* partial, int nblk, double* out, hipStream_t st) {
  const unsigned nb = stream_blocks(L) < (unsigned)nblk ? stream_blocks(L) : (unsigned)nblk;
  if (packable<T>(L, ld, Q, w))
    hipLaunchKernelGGL((k_axpy_norm_v<T>), dim3(nb), dim3(BLK), 0, st, w, Q, ld, k, h, L,
                       partial);
  else
    hipLaunchKernelGGL((k_axpy_norm<T>), dim3(nb), dim3(BLK), 0, st, w, Q, ld, k, h, L, partial);
  hipLaunchKernelGGL(k_reduce_rows, dim3(1), dim3(BLK), 0, st, partial, (int)nb, out);
  return hipGetLastError();
}

template <typename T>
hipError_t vec_axpy_multi(T* w, const T* Q, int64_t ld, int k, const double* h, double sign,
                          int64_t L, hipStream_t st) {
  if (packable<T>(L, ld, Q, w))
    hipLaunchKernelGGL((k_axpy_multi_v<T>), dim3(stream_blocks(L)), dim3(BLK), 0, st, w, Q, ld,
                       k, h, sign, L);
  else
    hipLaunchKernelGGL((k_axpy_multi<T>), dim3(stream_blocks(L)), dim3(BLK), 0, st, w, Q, ld, k,
                       h, sign, L);
  return hipGetLastError();
}

template <typename T>
hipError_t vec_scale(T* x, int64_t L, double s, hipStream_t st) {
  hipLaunchKernelGGL((k_scale<T>), dim3(stream_blocks(L)), dim3(BLK), 0, st, x, L, s);
  return hipGetLastError();
}

template <typename TD, typename TS>
hipError_t vec_copy_scaled(TD* dst, const TS* src, int64_t L, double s, hipStream_t st) {
  hipLaunchKernelGGL((k_copy_scaled<TD, TS>), dim3(stream_blocks(L)), dim3(BLK), 0, st, dst, src,
                     L, s);
  return hipGetLastError();
}

template <typename T>
hipError_t vec_scale_inv_norm(T* x, int64_t L, const double* nrm2, hipStream_t st) {
  hipLaunchKernelGGL((k_scale_inv_norm<T>), dim3(stream_blocks(L)), dim3(BLK), 0, st, x, L, nrm2);
  return hipGetLastError();
}

hipError_t inlet_speed(const double* d, int64_t n, int N, const int32_t* nodes, int64_t ni,
                       const double* tab, double* out, hipStream_t st) {
  if (ni <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_inlet_speed, dim3(N), dim3(BLK), 0, st, d, n, N, nodes, ni, tab, out);
  return hipGetLastError();
}

template <typename T>
hipError_t vec_zero(T* x, int64_t L, hipStream_t st) {
  hipLaunchKernelGGL((k_fill<T>), dim3(stream_blocks(L)), dim3(BLK), 0, st, x, L, 0.0);
  return hipGetLastError();
}

template <typename TU>
hipError_t vec_mul_dinv_add(double* y, const TU* u, const double* dinv, const uint8_t* dmask,
                            int64_t n, int N, int nch_y, int nch_u, double s, hipStream_t st) {
  hipLaunchKernelGGL((k_mul_dinv_add<TU>), dim3(blocks_for(n * 4 * N)), dim3(BLK), 0, st, y, u,
                     dinv, dmask, n, N, nch_y, nch_u, s);
  return hipGetLastError();
}

hipError_t channel_sum(const double* X, int64_t n, int nch, int N, int ch, double* out,
                       hipStream_t st) {
  hipError_t e = vec_zero<double>(out, N, st);
  if (e != hipSuccess || n == 0) return e;
  constexpr int64_t kChunk = 16384;
  const int64_t nch_ = (n + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(k_channel_sum, dim3(N, (unsigned)nch_), dim3(BLK), 0, st, X, n, nch, N, ch,
                     kChunk, out);
  return hipGetLastError();
}

hipError_t vec_blend(double* y, const double* a, const double* b, int64_t L, double alpha,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_blend, dim3(stream_blocks(L)), dim3(BLK), 0, st, y, a, b, L, alpha);
  return hipGetLastError();
}

hipError_t vec_nonfinite(const double* x, int64_t L, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_nonfinite, dim3(stream_blocks(L)), dim3(BLK), 0, st, x, L, flag);
  return hipGetLastError();
}

// explicit instantiations: FP64 everywhere, FP32 for the mixed-precision
// Krylov path (FP32 directions, accumulators and basis vectors).
#define HB_INST_IO(TI, TO)                                                                      \
  template hipError_t modal_to_samples<TI, TO>(const DevMesh&, int, const TI*, const double*,  \
                                               int, const double*, TO*, TO*, double*, int,      \
                                               hipStream_t);                                    \
  template hipError_t samples_to_modal<TI, TO>(const DevMesh&, int, const TI*, int, int, int,  \
                                               const double*, TO*, hipStream_t);                \
  template hipError_t prepare_direction<TI, TO>(const DevMesh&, int, const TI*, int,           \
                                                const double*, const double*, int,              \
                                                const double*, TO*, TO*, double*, int,          \
                                                hipStream_t);                                   \
  template hipError_t finish_rows<TI, TO>(const DevMesh&, int, const TI*, int, const double*,  \
                                          const TO*, TO*, hipStream_t);                         \
  template hipError_t vec_copy_scaled<TI, TO>(TI*, const TO*, int64_t, double, hipStream_t);
HB_INST_IO(double, double)
HB_INST_IO(double, float)
HB_INST_IO(float, float)
HB_INST_IO(float, double)
#undef HB_INST_IO

#define HB_INST_T(T)                                                                            \
  template hipError_t outlet_flux<T>(const DevMesh&, int, const T*, double*, hipStream_t);     \
  template hipError_t elem_jvp_exact<T>(const DevMesh&, const Phys&, const T*, const T*, T*,   \
                                        const ElemBlocks&, hipStream_t);                        \
  template hipError_t face_jvp<T>(const DevMesh&, const Phys&, const T*, const T*,             \
                                  const double*, const double*, T*, hipStream_t);               \
  template hipError_t vec_dots<T>(const T*, int64_t, int, const T*, int64_t, double*, int,     \
                                  double*, hipStream_t);                                        \
  template hipError_t vec_axpy_multi<T>(T*, const T*, int64_t, int, const double*, double,     \
                                        int64_t, hipStream_t);                                  \
  template hipError_t vec_mdots<T>(const T*, int64_t, int, const T*, int64_t, double*, int,    \
                                   double*, hipStream_t);                                       \
  template hipError_t vec_axpy_norm<T>(T*, const T*, int64_t, int, const double*, int64_t,      \
                                       double*, int, double*, hipStream_t);                     \
  template hipError_t vec_scale<T>(T*, int64_t, double, hipStream_t);                           \
  template hipError_t vec_scale_inv_norm<T>(T*, int64_t, const double*, hipStream_t);           \
  template hipError_t vec_zero<T>(T*, int64_t, hipStream_t);                                    \
  template hipError_t vec_mul_dinv_add<T>(double*, const T*, const double*, const uint8_t*,    \
                                          int64_t, int, int, int, double, hipStream_t);
HB_INST_T(double)
HB_INST_T(float)
#undef HB_INST_T

// ------------------------------------------------------------ time marching
// One generalized-alpha step at one time level: the state samples' H u
// channels hold (c1/dt) u_{n+1} (the time table's derivative entry); the
// step's history c1/dt u_n + (c1 - 1) a_n is subtracted so that they hold
// the acceleration at alpha_m.  S is node-major [a][7][1]; y_old [4][n]
// (velocity rows read) and a_old [3][n] are component-major.
__global__ void __launch_bounds__(256)
k_tm_history(int64_t n, double* __restrict__ S, const double* __restrict__ y_old,
             const double* __restrict__ a_old, double cu, double ca) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    S[a * NCH + 4 + i] -= cu * y_old[i * n + a] + ca * a_old[i * n + a];
}

hipError_t tm_history(const DevMesh& m, double* S, const double* y_old, const double* a_old,
                      double cu, double ca, hipStream_t st) {
  if (m.n == 0) return hipSuccess;
  const int64_t nb = (m.n + 255) / 256;
  hipLaunchKernelGGL(k_tm_history, dim3((unsigned)nb), dim3(256), 0, st, m.n, S, y_old, a_old,
                     cu, ca);
  return hipGetLastError();
}

// q(t) = a0 + sum_m a_m cos(m w t) + b_m sin(m w t) of the modal data
// d [3][2K+1][n] at one time t: out [3][n].
__global__ void __launch_bounds__(256)
k_modal_eval(int64_t n, int K, double omega, double t, const double* __restrict__ d,
             double* __restrict__ out) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const int N = 2 * K + 1;
  double v[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] = d[((int64_t)i * N) * n + a];
  for (int j = 1; j <= K; ++j) {
    double sn, cs;
    sincos((double)j * omega * t, &sn, &cs);
#pragma unroll
    for (int i = 0; i < 3; ++i)
      v[i] += cs * d[((int64_t)i * N + 2 * j - 1) * n + a] + sn * d[((int64_t)i * N + 2 * j) * n + a];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) out[(int64_t)i * n + a] = v[i];
}

// Mass-weighted squares of the velocity rows of y [4][n] and of a [3][n]:
// part[b] and part[nb + b] per workgroup b (grid-stride over nodes).
__global__ void __launch_bounds__(256)
k_tm_norms(int64_t n, const double* __restrict__ w, const double* __restrict__ y,
           const double* __restrict__ a, double* __restrict__ part) {
  __shared__ double su[256], sa[256];
  double u2 = 0.0, a2 = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    double pu = 0.0, pa = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double yu = y[(int64_t)i * n + k], ya = a[(int64_t)i * n + k];
      pu += yu * yu;
      pa += ya * ya;
    }
    u2 += w[k] * pu;
    a2 += w[k] * pa;
  }
  su[threadIdx.x] = u2;
  sa[threadIdx.x] = a2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      su[threadIdx.x] += su[threadIdx.x + s];
      sa[threadIdx.x] += sa[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = su[0];
    part[gridDim.x + blockIdx.x] = sa[0];
  }
}

// out[0..1] = sums of the two rows of part [2][nb] (one workgroup).
__global__ void __launch_bounds__(256)
k_tm_norms_sum(int nb, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double su[256], sa[256];
  double u2 = 0.0, a2 = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    u2 += part[b];
    a2 += part[nb + b];
  }
  su[threadIdx.x] = u2;
  sa[threadIdx.x] = a2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      su[threadIdx.x] += su[threadIdx.x + s];
      sa[threadIdx.x] += sa[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = su[0];
    out[1] = sa[0];
  }
}

// a_{n+1} = (u_{n+1} - u_n) / (gamma dt) with gamma = 1 (rho_inf = 0).
__global__ void __launch_bounds__(256)
k_tm_accel(int64_t n, const double* __restrict__ y_new, const double* __restrict__ y_old,
           double* __restrict__ a, double inv_dt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    a[(int64_t)i * n + k] = (y_new[(int64_t)i * n + k] - y_old[(int64_t)i * n + k]) * inv_dt;
}

hipError_t modal_eval(const DevMesh& m, int K, double omega, double t, const double* d,
                      double* out, hipStream_t st) {
  if (m.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_modal_eval, dim3((unsigned)((m.n + 255) / 256)), dim3(256), 0, st, m.n,
                     K, omega, t, d, out);
  return hipGetLastError();
}

hipError_t tm_norms(const DevMesh& m, const double* y, const double* a, double* part, int nb,
                    double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_tm_norms, dim3((unsigned)nb), dim3(256), 0, st, m.n, m.mass, y, a, part);
  hipLaunchKernelGGL(k_tm_norms_sum, dim3(1), dim3(256), 0, st, nb, (const double*)part, out);
  return hipGetLastError();
}

hipError_t tm_accel(const DevMesh& m, const double* y_new, const double* y_old, double* a,
                    double inv_dt, hipStream_t st) {
  if (m.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tm_accel, dim3((unsigned)((m.n + 255) / 256)), dim3(256), 0, st, m.n,
                     y_new, y_old, a, inv_dt);
  return hipGetLastError();
}

}  // namespace hb
