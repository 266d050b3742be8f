// Internal declarations shared by the kernel and host translation units of
// the HB library.  Not part of the public interface (see include/hb.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace hb {

// Thread-local message returned by hb_last_error().
void set_last_error(const std::string& msg);

// Owning device array of T (grown on demand, freed on destruction).
template <class T>
struct DeviceArray {
  T* p = nullptr;
  size_t n = 0;
  DeviceArray() = default;
  DeviceArray(const DeviceArray&) = delete;
  DeviceArray& operator=(const DeviceArray&) = delete;
  DeviceArray(DeviceArray&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  ~DeviceArray() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  hipError_t ensure(size_t count) {
    if (p && count <= n) return hipSuccess;
    release();
    hipError_t e = hipMalloc((void**)&p, sizeof(T) * (count ? count : 1));
    if (e == hipSuccess) n = count;
    return e;
  }
  size_t bytes() const { return sizeof(T) * n; }
};

// Library-owned device view of a mesh (structure of arrays).
struct DevMesh {
  int64_t n = 0;      // nodes
  int64_t ne = 0;     // tetrahedra
  int64_t nof = 0;    // outlet triangles
  int32_t n_out = 0;  // outlet groups
  const int32_t* tets = nullptr;  // [4][ne]
  const double* geo = nullptr;    // [GEO_COUNT][ne]
  const uint8_t* dmask = nullptr; // [n] 1 on Dirichlet nodes
  const int32_t* of = nullptr;    // [3][nof] outlet triangle nodes
  const double* ofn = nullptr;    // [4][nof] unit outward normal, area
  const int32_t* oid = nullptr;   // [nof] outlet index
  const double* mass = nullptr;   // [n] diagonal of the consistent mass, int N_A^2
};

// Element blocks for workgroup-level accumulation: consecutive runs of
// `size` tetrahedra, the unique nodes of each run, and every element node's
// slot among them.
struct ElemBlocks {
  int32_t size = 0;
  int32_t max_unique = 0;
  const int32_t* ptr = nullptr;    // [n_blocks + 1] offsets into nodes
  const int32_t* nodes = nullptr;  // unique nodes of each block
  const uint8_t* slot = nullptr;   // [4][ne] slot of element node A in its block
};

// Per-tetrahedron geometry rows: gradients of N_1..N_3, volume, the upper
// triangle of xi = J^-T J^-1, xi:xi, and grad N_0 = -sum of the others.
enum {
  GEO_G1 = 0, GEO_G2 = 3, GEO_G3 = 6, GEO_V = 9,
  GEO_XI00 = 10, GEO_XI01 = 11, GEO_XI02 = 12, GEO_XI11 = 13, GEO_XI12 = 14, GEO_XI22 = 15,
  GEO_XIXI = 16,
  GEO_G0 = 17,  // grad N_0 = -(grad N_1 + grad N_2 + grad N_3), stored for the quad-lane kernels
  GEO_COUNT = 20
};

struct Phys {
  double rho, mu, nu, C_I, beta, omega;
  double inv_rho;    // 1 / rho
  double tau_add;    // added inside tau's bracket: 0 for HB, omega-hat^2 for a marched step
  double shift;      // pseudo-time mass coefficient on velocity rows (0 = none)
  const double* shift_dev;  // if set, the exact-Jv kernel reads the shift here instead
                            // (replayed graphs stay valid when the shift changes)
  int32_t N;
  int32_t backflow;  // 1 = backflow term on outlets
};

// Time-axis tables, each N x N doubles, stored consecutively.
enum {
  TAB_BINV = 0,  // [s][m] samples = Binv . modal
  TAB_BDER = 1,  // [s][m] d/dt samples = Bder . modal
  TAB_FWD = 2,   // [m][s] modal = Fwd . samples
  TAB_FWDD = 3,  // [m][s] modal(H x) = FwdD . samples(x)
  TAB_H = 4,     // [s][k] H in samples
  TAB_COUNT = 5
};

// Samples buffers are node-major: X[a][c][s] with c a channel.  The state
// and direction buffers carry 7 channels (u1 u2 u3 p Hu1 Hu2 Hu3); the
// element accumulator carries 7 channels (r^m_1..3, r^c, z_1..3); Krylov
// vectors carry 4 channels.
constexpr int NCH = 7;

// Launchers.  Templates are instantiated for double, and for float where
// the mixed-precision Krylov path needs them (directions, accumulators and
// basis vectors in FP32; state, residual and preconditioner in FP64).
template <typename TI, typename TO>
hipError_t modal_to_samples(const DevMesh& m, int N, const TI* Y, const double* dir,
                            int zero_dirichlet, const double* tab, TO* S, TO* acc_zero,
                            double* q_zero, int nq, hipStream_t st);
template <typename TA, typename TO>
hipError_t samples_to_modal(const DevMesh& m, int N, const TA* acc, int use_z, int zero_dir_rows,
                            int in_ch, const double* tab, TO* R, hipStream_t st);
template <typename R>
hipError_t outlet_flux(const DevMesh& m, int N, const R* S, double* Q, hipStream_t st);
hipError_t elem_residual(const DevMesh& m, const Phys& p, const double* S, double* acc,
                         const ElemBlocks& eb, hipStream_t st);
template <typename R>
hipError_t elem_jvp_exact(const DevMesh& m, const Phys& p, const R* Sy, const R* Sv, R* acc,
                          const ElemBlocks& eb, hipStream_t st);
hipError_t elem_jvp_paper(const DevMesh& m, const Phys& p, const double* Sy, const double* Sv,
                          double* acc, hipStream_t st);
hipError_t elem_jacobi(const DevMesh& m, const Phys& p, const double* Sy, double* dg,
                       int time_terms, hipStream_t st);
hipError_t face_residual(const DevMesh& m, const Phys& p, const double* S, const double* hs,
                         const double* Rk, const double* Q, double* acc, hipStream_t st);
template <typename R>
hipError_t face_jvp(const DevMesh& m, const Phys& p, const R* Sy, const R* Sv, const double* Rk,
                    const double* dQ, R* acc, hipStream_t st);
hipError_t jacobi_out(const DevMesh& m, int N, int nc, const double* dg, double* D, double* dinv,
                      hipStream_t st);
// sample-space nodal passes (Krylov path)
template <typename TQ, typename TS>
hipError_t prepare_direction(const DevMesh& m, int N, const TQ* q, int in_ch, const double* dinv,
                             const double* binv, int zero_dirichlet, const double* tab, TS* Sv,
                             TS* acc_zero, double* q_zero, int nq, hipStream_t st);
// Per-node velocity time blocks of the exact Jacobian's nodal diagonal,
// inverted in place: binv[a][s][k]; identity at Dirichlet nodes; dg with
// 4 channels (K, L, T, X) from elem_jacobi(time_terms = 1).
hipError_t block_factor(const DevMesh& m, int N, const double* dg, const double* mass,
                        double rho, const double* tab, double* binv, hipStream_t st);
template <typename TA, typename TO>
hipError_t finish_rows(const DevMesh& m, int N, const TA* acc, int use_z, const double* tab,
                       const TO* id_rows, TO* out, hipStream_t st);
// vectors
template <typename T>
hipError_t vec_dots(const T* Q, int64_t ld, int k, const T* w, int64_t L, double* partial,
                    int nblk, double* out, hipStream_t st);
template <typename T>
hipError_t vec_axpy_multi(T* w, const T* Q, int64_t ld, int k, const double* h, double sign,
                          int64_t L, hipStream_t st);
// out[j] = Q_j . w, j < k (one partial-sum launch for all j, one reduction;
// partial: k rows of nblk doubles)
template <typename T>
hipError_t vec_mdots(const T* Q, int64_t ld, int k, const T* w, int64_t L, double* partial,
                     int nblk, double* out, hipStream_t st);
// w -= sum_j h_j Q_j; out[0] = |w|^2 of the result (partial: nblk doubles)
template <typename T>
hipError_t vec_axpy_norm(T* w, const T* Q, int64_t ld, int k, const double* h, int64_t L,
                         double* partial, int nblk, double* out, hipStream_t st);
template <typename T>
hipError_t vec_scale(T* x, int64_t L, double s, hipStream_t st);
template <typename TD, typename TS>
hipError_t vec_copy_scaled(TD* dst, const TS* src, int64_t L, double s, hipStream_t st);
template <typename T>
hipError_t vec_zero(T* x, int64_t L, hipStream_t st);
// x /= sqrt(*nrm2) (device scalar) when positive and finite
template <typename T>
hipError_t vec_scale_inv_norm(T* x, int64_t L, const double* nrm2, hipStream_t st);
// out[s] = mean |u(t_s)| over the given inlet nodes of the modal Dirichlet data
hipError_t inlet_speed(const double* d, int64_t n, int N, const int32_t* nodes, int64_t ni,
                       const double* tab, double* out, hipStream_t st);
template <typename TU>
hipError_t vec_mul_dinv_add(double* y, const TU* u, const double* dinv, const uint8_t* dmask,
                            int64_t n, int N, int nch_y, int nch_u, double s, hipStream_t st);
hipError_t vec_nonfinite(const double* x, int64_t L, int* flag, hipStream_t st);
// out[s] = sum over nodes a of X[a][ch][s] (X [n][nch][N]); out [N] device
hipError_t channel_sum(const double* X, int64_t n, int nch, int N, int ch, double* out,
                       hipStream_t st);
// y = a + alpha (b - a); y may alias a or b
hipError_t vec_blend(double* y, const double* a, const double* b, int64_t L, double alpha,
                     hipStream_t st);
// Mean-flow modal preconditioner (hb_precond.hip): per-mode complex systems
// of the sample-averaged frozen tangent, approximated by aggregation
// multigrid V-cycles on the node graph.
struct Precond;
// pairwise = 1: aggregates from two passes of pairwise matching (up to 4
// nodes); 0: a node and its free neighbours.
hipError_t precond_create(int64_t n, int64_t ne, const int32_t* tets_dev, int coarse_max,
                          int pairwise, Precond** out);
void precond_destroy(Precond* p);
size_t precond_bytes(const Precond* p);
// sizes[l] = nodes of level l (l < max); returns the number of levels
int precond_levels(const Precond* p, int64_t* sizes, int max);
// Coefficients at the state samples Sy ([n][7][N]) with pseudo-time mass
// coefficient sigma; nu Jacobi sweeps (weight wj) before and after each
// coarse correction (weight gamma), `cycles` cycles per application;
// smoother 0 damped block Jacobi, 1 symmetric block Gauss-Seidel (colour
// classes; wj unused); wcycle 1 for W-cycles; fp32 1 for cycles on FP32
// vectors and coefficients (the coarsest inverse stays FP64).
hipError_t precond_setup(Precond* pc, const DevMesh& m, const Phys& p, const double* Sy,
                         double sigma, int nu, int cycles, double wj, double gamma, int smoother,
                         int wcycle, int fp32, hipStream_t st);
// z [n][4][N] = M^-1 q, q with in_ch channels per node ([n][in_ch][N]).
template <typename TQ, typename TZ>
hipError_t precond_apply(Precond* pc, int64_t n, const TQ* q, int in_ch, TZ* z, hipStream_t st);
// z [n][4][N] = M q (the mean-flow operator itself, for checking).
template <typename TQ, typename TZ>
hipError_t precond_matvec(Precond* pc, int64_t n, const TQ* q, int in_ch, TZ* z, hipStream_t st);
// 1 in *flag_host if the coarsest-level inversion met a zero pivot (waits).
hipError_t precond_singular(Precond* pc, int* flag_host, hipStream_t st);

// Time-marching step: S[a][4+i][0] -= cu y_old[i][a] + ca a_old[i][a] (N = 1).
hipError_t tm_history(const DevMesh& m, double* S, const double* y_old, const double* a_old,
                      double cu, double ca, hipStream_t st);
// out [3][n] = modal data d [3][2K+1][n] evaluated at time t.
hipError_t modal_eval(const DevMesh& m, int K, double omega, double t, const double* d,
                      double* out, hipStream_t st);
// out[0] = sum_a mass_a |u_a|^2 (velocity rows of y [4][n]), out[1] = the same
// of a [3][n]; part holds 2 nb doubles (nb workgroups, nb >= 1).
hipError_t tm_norms(const DevMesh& m, const double* y, const double* a, double* part, int nb,
                    double* out, hipStream_t st);
// a [3][n] = (velocity rows of y_new - y_old) * inv_dt.
hipError_t tm_accel(const DevMesh& m, const double* y_new, const double* y_old, double* a,
                    double inv_dt, hipStream_t st);

}  // namespace hb
