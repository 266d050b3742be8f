// Host side of the HB library: mesh handles, argument checking, workspace,
// the modal residual / Jacobian-vector entry points and the Newton-GMRES
// driver (Section 2.3 of arXiv 2411.14315).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "hb.h"
#include "hb_internal.h"

using hb::DevMesh;
using hb::Phys;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

}  // namespace

void hb::set_last_error(const std::string& msg) { g_err = msg; }

namespace {

#define HB_CHECK(...)                                                               \
  do {                                                                              \
    hipError_t e_ = (__VA_ARGS__);                                                  \
    if (e_ != hipSuccess)                                                           \
      return fail(e_ == hipErrorOutOfMemory ? HB_ERR_OOM : HB_ERR_DEVICE,           \
                  std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_));        \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t ensure(size_t b) {
    if (b <= bytes && p) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, b ? b : 8);
    if (e == hipSuccess) bytes = b;
    return e;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Buffers that depend on the number of samples N.
struct Workspace {
  int N = -1;
  DevBuf Sy, Sv, acc, tab, small, dg, dinv, binv;
  DevBuf Sy32, Sv32, acc32;  // FP32 state copy, direction and accumulator (mixed precision)
  std::vector<double> tab_host;
  std::vector<double> bc_host;  // hs (n_out N) then R (n_out), as last uploaded
  bool bc_has_R = false;
  bool bc_valid = false;
};

}  // namespace

// Krylov buffers kept on the mesh between solves, pinned host slots for the
// Arnoldi coefficients, and events.
struct SolverBufs {
  DevBuf basis, xvec, rvec, tmp, partial, hdev, rbuf, uc, shift, sysave, syfull;
  double* hpin = nullptr;  // pinned host copies of each Arnoldi step's coefficients
  size_t hpin_n = 0;
  hipEvent_t evh[2] = {};  // Arnoldi step completion (ping-pong)
  hipEvent_t evj[6] = {};  // operator timing: two (start, after preconditioner, end) triples
  // Arnoldi steps captured as HIP graphs, one per step index, valid while
  // every pointer and size they were captured with (key) is unchanged.
  std::vector<uintptr_t> gkey;
  std::vector<hipGraphExec_t> gexec;
  hipStream_t gstream = nullptr;  // private stream used only for capture
  void drop_graphs() {
    for (auto& e : gexec)
      if (e) (void)hipGraphExecDestroy(e);
    gexec.clear();
    gkey.clear();
  }
  ~SolverBufs() {
    drop_graphs();
    if (gstream) (void)hipStreamDestroy(gstream);
    if (hpin) (void)hipHostFree(hpin);
    for (auto& e : evh)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : evj)
      if (e) (void)hipEventDestroy(e);
  }
};

struct BlockMap {
  hb::ElemBlocks eb;
  DevBuf ptr, nodes, slot;
};

struct hb_mesh {
  DevMesh dm;
  BlockMap bmaps[4];  // element blocks of 32, 16, 8 and 4 tetrahedra
  DevBuf tets, geo, dmask, of, ofn, oid, mass;
  int64_t n_dirichlet = 0, n_reoriented = 0, n_inlet = 0;
  std::vector<int32_t> inlet_nodes;  // inlet nodes that are not wall nodes
  DevBuf inlet_dev;                  // the same list on the device
  double mean_vol = 0.0;
  int device = 0;
  Workspace ws;
  SolverBufs sb;
  DevBuf tm_yold, tm_g, tm_part;  // time marching: previous state, boundary data, norms
  hb::Precond* pc = nullptr;       // mean-flow preconditioner hierarchy (built on first use)
  int pc_coarse_max = 0, pc_pairwise = -1;
  DevBuf pcz;                      // preconditioned vector [n][4][N]
  // stage timing (hb_set_timing)
  bool timing = false;
  bool timed_call = false;
  hipEvent_t ev[7] = {};
  ~hb_mesh() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    hb::precond_destroy(pc);
  }
  size_t bytes_held() const {
    size_t b = 0;
    for (const DevBuf* d : {&tets, &geo, &dmask, &of, &ofn, &oid, &mass, &inlet_dev, &ws.Sy, &ws.Sv,
                            &ws.acc, &ws.tab, &ws.small, &ws.dg, &ws.dinv, &ws.binv, &ws.Sy32,
                            &ws.Sv32, &ws.acc32, &sb.basis, &sb.xvec, &sb.rvec, &sb.tmp,
                            &sb.partial, &sb.hdev, &sb.rbuf, &sb.uc, &sb.shift, &sb.sysave, &sb.syfull, &tm_yold, &tm_g,
                            &tm_part})
      b += d->bytes;
    for (const auto& bm : bmaps) b += bm.ptr.bytes + bm.nodes.bytes + bm.slot.bytes;
    b += pcz.bytes + hb::precond_bytes(pc);
    return b;
  }
};

namespace {

// Real DFT tables for N = 2K+1 samples t_n = n T/N (Section 2.1,
// eq. upghdft, in the real [a_0, a_1, b_1, ...] ordering).
void build_tables(int K, double omega, std::vector<double>& tab) {
  const int N = 2 * K + 1;
  const size_t NN = (size_t)N * N;
  tab.assign(hb::TAB_COUNT * NN, 0.0);
  double* Binv = tab.data() + hb::TAB_BINV * NN;
  double* Bder = tab.data() + hb::TAB_BDER * NN;
  double* Fwd = tab.data() + hb::TAB_FWD * NN;
  double* FwdD = tab.data() + hb::TAB_FWDD * NN;
  double* Hs = tab.data() + hb::TAB_H * NN;
  const double two_pi = 6.283185307179586476925286766559;
  for (int s = 0; s < N; ++s) {
    Binv[s * N + 0] = 1.0;
    Fwd[0 * N + s] = 1.0 / N;
    for (int j = 1; j <= K; ++j) {
      const double th = two_pi * (double)((j * s) % N) / (double)N;
      const double c = std::cos(th), sn = std::sin(th);
      Binv[s * N + 2 * j - 1] = c;
      Binv[s * N + 2 * j] = sn;
      Bder[s * N + 2 * j - 1] = -j * omega * sn;
      Bder[s * N + 2 * j] = j * omega * c;
      Fwd[(2 * j - 1) * N + s] = 2.0 * c / N;
      Fwd[(2 * j) * N + s] = 2.0 * sn / N;
      // D (a_j, b_j) = (j w b_j, -j w a_j)
      FwdD[(2 * j - 1) * N + s] = j * omega * 2.0 * sn / N;
      FwdD[(2 * j) * N + s] = -j * omega * 2.0 * c / N;
    }
  }
  for (int s = 0; s < N; ++s)
    for (int k = 0; k < N; ++k) {
      double v = 0.0;
      for (int m = 0; m < N; ++m) v += Bder[s * N + m] * Fwd[m * N + k];
      Hs[s * N + k] = v;
    }
}

int check_params(const hb_params* prm) {
  if (!prm) return fail(HB_ERR_ARG, "params is NULL");
  if (!(prm->rho > 0) || !(prm->mu > 0) || !(prm->period > 0))
    return fail(HB_ERR_ARG, "rho, mu and period must be positive");
  if (prm->K < 0 || prm->K > 32) return fail(HB_ERR_ARG, "K must be in 0..32");
  if (!(prm->C_I > 0)) return fail(HB_ERR_ARG, "C_I must be positive");
  if (!(prm->beta_bf >= 0)) return fail(HB_ERR_ARG, "beta_bf must be >= 0");
  return HB_OK;
}

Phys make_phys(const hb_params* prm, double shift) {
  Phys p;
  p.rho = prm->rho;
  p.mu = prm->mu;
  p.nu = prm->mu / prm->rho;
  p.inv_rho = 1.0 / prm->rho;
  p.C_I = prm->C_I;
  p.beta = prm->beta_bf;
  p.omega = 6.283185307179586476925286766559 / prm->period;
  p.tau_add = 0.0;
  p.shift = shift;
  p.shift_dev = nullptr;
  p.N = 2 * prm->K + 1;
  p.backflow = prm->beta_bf > 0 ? 1 : 0;
  return p;
}

// Make workspace ready for N samples and the boundary data of bc.
int prepare(hb_mesh* m, const hb_params* prm, const hb_bc* bc, hipStream_t st) {
  int rc = check_params(prm);
  if (rc) return rc;
  if (!bc || !bc->dirichlet) return fail(HB_ERR_ARG, "bc.dirichlet is NULL");
  Workspace& w = m->ws;
  const int N = 2 * prm->K + 1;
  const int64_t n = m->dm.n;
  const int nout = m->dm.n_out;
  if (w.N != N) {
    HB_CHECK(w.Sy.ensure(sizeof(double) * n * hb::NCH * N));
    HB_CHECK(w.Sv.ensure(sizeof(double) * n * hb::NCH * N));
    HB_CHECK(w.acc.ensure(sizeof(double) * n * hb::NCH * N));
    HB_CHECK(w.dg.ensure(sizeof(double) * n * 4 * N));
    HB_CHECK(w.dinv.ensure(sizeof(double) * n * 2 * N));
    HB_CHECK(w.tab.ensure(sizeof(double) * hb::TAB_COUNT * N * N));
    // small: Q, dQ, hs (n_out N each), R (n_out), flag
    HB_CHECK(w.small.ensure(sizeof(double) * (3 * (size_t)nout * N + nout + 8)));
    w.N = N;
    w.bc_valid = false;
    w.tab_host.clear();
  }
  std::vector<double> tab;
  build_tables(prm->K, 6.283185307179586476925286766559 / prm->period, tab);
  if (tab != w.tab_host) {
    w.tab_host = tab;
    HB_CHECK(hipMemcpyAsync(w.tab.p, w.tab_host.data(), sizeof(double) * tab.size(),
                            hipMemcpyHostToDevice, st));
  }
  // outlet traction samples h_n (from modal coefficients) and resistances
  std::vector<double> bch((size_t)nout * N + nout, 0.0);
  if (bc->outlet_h) {
    const double* Binv = tab.data() + hb::TAB_BINV * (size_t)N * N;
    for (int k = 0; k < nout; ++k)
      for (int s = 0; s < N; ++s) {
        double v = 0.0;
        for (int mm = 0; mm < N; ++mm) v += Binv[s * N + mm] * bc->outlet_h[(size_t)k * N + mm];
        bch[(size_t)k * N + s] = v;
      }
  }
  if (bc->outlet_R)
    for (int k = 0; k < nout; ++k) {
      if (!std::isfinite(bc->outlet_R[k])) return fail(HB_ERR_ARG, "non-finite outlet_R");
      bch[(size_t)nout * N + k] = bc->outlet_R[k];
    }
  const bool hasR = bc->outlet_R != nullptr;
  if (!w.bc_valid || hasR != w.bc_has_R || bch != w.bc_host) {
    w.bc_host = bch;
    w.bc_has_R = hasR;
    w.bc_valid = true;
    double* hs = w.small.as<double>() + 2 * (size_t)nout * N;
    if (!bch.empty())
      HB_CHECK(hipMemcpyAsync(hs, w.bc_host.data(), sizeof(double) * bch.size(),
                              hipMemcpyHostToDevice, st));
  }
  return HB_OK;
}

// Stage boundary k (0..6) of a timed call.
hipError_t mark(hb_mesh* m, int k, hipStream_t st) {
  if (!m->timing) return hipSuccess;
  if (k == 0) m->timed_call = true;
  return hipEventRecord(m->ev[k], st);
}

struct Ptrs {
  double* Q;
  double* dQ;
  const double* hs;
  const double* R;
  int* flag;
};

Ptrs small_ptrs(hb_mesh* m) {
  const int N = m->ws.N;
  const int nout = m->dm.n_out;
  double* b = m->ws.small.as<double>();
  Ptrs p;
  p.Q = b;
  p.dQ = b + (size_t)nout * N;
  p.hs = b + 2 * (size_t)nout * N;
  p.R = m->ws.bc_has_R ? b + 3 * (size_t)nout * N : nullptr;
  p.flag = reinterpret_cast<int*>(b + 3 * (size_t)nout * N + nout);
  return p;
}

int ensure_f32(hb_mesh* m) {
  Workspace& w = m->ws;
  const size_t b = sizeof(float) * (size_t)m->dm.n * hb::NCH * w.N;
  HB_CHECK(w.Sy32.ensure(b));
  HB_CHECK(w.Sv32.ensure(b));
  HB_CHECK(w.acc32.ensure(b));
  return HB_OK;
}

#ifndef HB_LDS_BUDGET
#define HB_LDS_BUDGET (64 * 1024)
#endif
// Largest element block whose LDS accumulator (unique nodes x 7 x N FP64
// values, in every precision) stays within the LDS budget per workgroup.
const hb::ElemBlocks& pick_blocks(const hb_mesh* m, int N, size_t elem = sizeof(double)) {
  for (const auto& b : m->bmaps)
    if ((size_t)b.eb.max_unique * hb::NCH * N * elem <= HB_LDS_BUDGET) return b.eb;
  return m->bmaps[3].eb;
}

// Unique nodes of each run of `size` consecutive tetrahedra and the slot of
// every element node among them.
int build_blocks(BlockMap& bm, const std::vector<int32_t>& T, int64_t ne, int size) {
  const int64_t nb = (ne + size - 1) / size;
  std::vector<int32_t> ptr(nb + 1, 0), nodes;
  std::vector<uint8_t> slot(4 * ne);
  nodes.reserve(ne * 2);
  int maxu = 0;
  std::vector<int32_t> u;
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t e0 = b * size, e1 = std::min<int64_t>(ne, e0 + size);
    u.assign(T.begin() + 4 * e0, T.begin() + 4 * e1);
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    for (int64_t t = e0; t < e1; ++t)
      for (int A = 0; A < 4; ++A)
        slot[A * ne + t] =
            (uint8_t)(std::lower_bound(u.begin(), u.end(), T[4 * t + A]) - u.begin());
    nodes.insert(nodes.end(), u.begin(), u.end());
    ptr[b + 1] = (int32_t)nodes.size();
    maxu = std::max<int>(maxu, (int)u.size());
  }
  HB_CHECK(bm.ptr.ensure(sizeof(int32_t) * ptr.size()));
  HB_CHECK(bm.nodes.ensure(sizeof(int32_t) * nodes.size()));
  HB_CHECK(bm.slot.ensure(slot.size()));
  HB_CHECK(hipMemcpy(bm.ptr.p, ptr.data(), sizeof(int32_t) * ptr.size(), hipMemcpyHostToDevice));
  HB_CHECK(hipMemcpy(bm.nodes.p, nodes.data(), sizeof(int32_t) * nodes.size(),
                     hipMemcpyHostToDevice));
  HB_CHECK(hipMemcpy(bm.slot.p, slot.data(), slot.size(), hipMemcpyHostToDevice));
  bm.eb.size = size;
  bm.eb.max_unique = maxu;
  bm.eb.ptr = bm.ptr.as<int32_t>();
  bm.eb.nodes = bm.nodes.as<int32_t>();
  bm.eb.slot = bm.slot.as<uint8_t>();
  return HB_OK;
}

// The mean-flow preconditioner's hierarchy for this mesh (built once per
// coarse-level size) and its output buffer for N samples.
int ensure_precond(hb_mesh* m, int coarse_max, int pairwise, int N) {
  if (!m->pc || m->pc_coarse_max != coarse_max || m->pc_pairwise != pairwise) {
    hb::precond_destroy(m->pc);
    m->pc = nullptr;
    const hipError_t e = hb::precond_create(m->dm.n, m->dm.ne, m->dm.tets, coarse_max, pairwise,
                                            &m->pc);
    if (e == hipErrorInvalidValue)
      return fail(HB_ERR_ARG, "the multigrid hierarchy does not coarsen below 2048 nodes");
    HB_CHECK(e);
    m->pc_coarse_max = coarse_max;
    m->pc_pairwise = pairwise;
  }
  HB_CHECK(m->pcz.ensure(sizeof(double) * (size_t)m->dm.n * 4 * N));
  return HB_OK;
}

constexpr int kCoarseMax = 24;

}  // namespace

extern "C" {

const char* hb_last_error(void) { return g_err.c_str(); }

int hb_mesh_create(int64_t n_nodes, const double* xyz, int64_t n_tets, const int32_t* tets,
                   int64_t n_faces, const int32_t* faces, const int32_t* face_group,
                   int32_t n_groups, const int32_t* group_kind, hb_mesh** out) {
  if (!out) return fail(HB_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n_nodes <= 0 || n_tets <= 0 || n_faces < 0 || n_groups <= 0)
    return fail(HB_ERR_ARG, "sizes must be positive");
  if (n_nodes > INT32_MAX) return fail(HB_ERR_ARG, "more than 2^31-1 nodes");
  if (!xyz || !tets || (n_faces > 0 && (!faces || !face_group)) || !group_kind)
    return fail(HB_ERR_ARG, "NULL mesh array");
  int n_outlets = 0;
  for (int g = 0; g < n_groups; ++g) {
    if (group_kind[g] < HB_WALL || group_kind[g] > HB_OUTLET)
      return fail(HB_ERR_ARG, "group_kind out of range");
    n_outlets += group_kind[g] == HB_OUTLET;
  }
  if (n_outlets == 0) return fail(HB_ERR_ARG, "no outlet group: pressure undetermined");
  if (n_outlets > 64) return fail(HB_ERR_ARG, "more than 64 outlet groups");
  for (int64_t i = 0; i < 3 * n_nodes; ++i)
    if (!std::isfinite(xyz[i])) return fail(HB_ERR_MESH, "non-finite coordinate");

  std::vector<int32_t> T(tets, tets + 4 * n_tets);
  for (int64_t i = 0; i < 4 * n_tets; ++i)
    if (T[i] < 0 || T[i] >= n_nodes) return fail(HB_ERR_MESH, "tetrahedron node index out of range");
  for (int64_t f = 0; f < n_faces; ++f) {
    for (int k = 0; k < 3; ++k)
      if (faces[3 * f + k] < 0 || faces[3 * f + k] >= n_nodes)
        return fail(HB_ERR_MESH, "face node index out of range");
    if (face_group[f] < 0 || face_group[f] >= n_groups)
      return fail(HB_ERR_MESH, "face group out of range");
  }

  auto P = [&](int32_t a, int k) { return xyz[3 * (int64_t)a + k]; };
  const int64_t ne = n_tets;
  std::vector<double> geo((size_t)hb::GEO_COUNT * ne);
  std::vector<double> vol(ne);
  int64_t reoriented = 0;
  double vsum = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int64_t t = 0; t < ne; ++t) {
      int32_t* v = &T[4 * t];
      double J[3][3];  // columns x_k - x_0
      for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) J[i][k] = P(v[k + 1], i) - P(v[0], i);
      const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                       - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                       + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      if (pass == 0) {
        if (det < 0) {
          std::swap(v[2], v[3]);
          ++reoriented;
          vol[t] = -det / 6.0;
        } else {
          vol[t] = det / 6.0;
        }
        vsum += vol[t];
        continue;
      }
      // inverse: row k of J^-1 = gradient of barycentric coordinate k+1
      double Ji[3][3];
      Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
      Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
      Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
      Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
      Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
      Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
      Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
      Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
      Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
      for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) geo[(size_t)(hb::GEO_G1 + 3 * k + i) * ne + t] = Ji[k][i];
      for (int i = 0; i < 3; ++i)
        geo[(size_t)(hb::GEO_G0 + i) * ne + t] = -(Ji[0][i] + Ji[1][i] + Ji[2][i]);
      geo[(size_t)hb::GEO_V * ne + t] = det / 6.0;
      double xi[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          xi[i][j] = Ji[0][i] * Ji[0][j] + Ji[1][i] * Ji[1][j] + Ji[2][i] * Ji[2][j];
      geo[(size_t)hb::GEO_XI00 * ne + t] = xi[0][0];
      geo[(size_t)hb::GEO_XI01 * ne + t] = xi[0][1];
      geo[(size_t)hb::GEO_XI02 * ne + t] = xi[0][2];
      geo[(size_t)hb::GEO_XI11 * ne + t] = xi[1][1];
      geo[(size_t)hb::GEO_XI12 * ne + t] = xi[1][2];
      geo[(size_t)hb::GEO_XI22 * ne + t] = xi[2][2];
      double xx = 0.0;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) xx += xi[i][j] * xi[i][j];
      geo[(size_t)hb::GEO_XIXI * ne + t] = xx;
    }
    if (pass == 0) {
      const double vmean = vsum / ne;
      for (int64_t t = 0; t < ne; ++t)
        if (!(vol[t] >= 1e-14 * vmean)) return fail(HB_ERR_MESH, "degenerate tetrahedron");
    }
  }

  // node classes: Dirichlet = nodes of wall and inlet faces
  std::vector<uint8_t> dmask(n_nodes, 0), wall(n_nodes, 0), inlet(n_nodes, 0);
  std::vector<int32_t> gid2out(n_groups, -1);
  {
    int k = 0;
    for (int g = 0; g < n_groups; ++g)
      if (group_kind[g] == HB_OUTLET) gid2out[g] = k++;
  }
  std::vector<int64_t> ofaces;
  for (int64_t f = 0; f < n_faces; ++f) {
    const int kind = group_kind[face_group[f]];
    for (int k = 0; k < 3; ++k) {
      const int32_t a = faces[3 * f + k];
      if (kind == HB_WALL) wall[a] = 1;
      if (kind == HB_INLET) inlet[a] = 1;
      if (kind != HB_OUTLET) dmask[a] = 1;
    }
    if (kind == HB_OUTLET) ofaces.push_back(f);
  }
  const int64_t nof = (int64_t)ofaces.size();

  // outlet faces: find the owning tetrahedron, orient the normal outwards
  using Key = std::array<int32_t, 3>;
  std::vector<std::pair<Key, int64_t>> keys(nof);
  for (int64_t i = 0; i < nof; ++i) {
    const int32_t* fv = faces + 3 * ofaces[i];
    Key k = {fv[0], fv[1], fv[2]};
    std::sort(k.begin(), k.end());
    keys[i] = {k, i};
  }
  std::sort(keys.begin(), keys.end());
  std::vector<int32_t> opp(nof, -1);
  static const int loc[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
  if (nof > 0)
    for (int64_t t = 0; t < ne; ++t)
      for (int lf = 0; lf < 4; ++lf) {
        Key k = {T[4 * t + loc[lf][0]], T[4 * t + loc[lf][1]], T[4 * t + loc[lf][2]]};
        std::sort(k.begin(), k.end());
        auto it = std::lower_bound(keys.begin(), keys.end(), std::make_pair(k, (int64_t)-1));
        for (; it != keys.end() && it->first == k; ++it) opp[it->second] = T[4 * t + lf];
      }
  std::vector<int32_t> ofv(3 * nof), oid(nof);
  std::vector<double> ofn(4 * nof);
  for (int64_t i = 0; i < nof; ++i) {
    if (opp[i] < 0) return fail(HB_ERR_MESH, "outlet face is not a face of any tetrahedron");
    const int32_t* fv = faces + 3 * ofaces[i];
    double a[3], b[3], c[3], nrm[3];
    for (int k = 0; k < 3; ++k) {
      a[k] = P(fv[1], k) - P(fv[0], k);
      b[k] = P(fv[2], k) - P(fv[0], k);
      c[k] = P(opp[i], k) - P(fv[0], k);
    }
    nrm[0] = a[1] * b[2] - a[2] * b[1];
    nrm[1] = a[2] * b[0] - a[0] * b[2];
    nrm[2] = a[0] * b[1] - a[1] * b[0];
    double sgn = nrm[0] * c[0] + nrm[1] * c[1] + nrm[2] * c[2];
    const double len = std::sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
    if (!(len > 0)) return fail(HB_ERR_MESH, "degenerate outlet face");
    const double s = sgn > 0 ? -1.0 / len : 1.0 / len;
    for (int k = 0; k < 3; ++k) {
      ofv[k * nof + i] = fv[k];
      ofn[k * nof + i] = nrm[k] * s;
    }
    ofn[3 * nof + i] = 0.5 * len;
    oid[i] = gid2out[face_group[ofaces[i]]];
  }

  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count == 0)
    return fail(HB_ERR_DEVICE, "no HIP device");
  std::unique_ptr<hb_mesh> m(new hb_mesh());
  (void)hipGetDevice(&m->device);
  std::vector<int32_t> Tsoa(4 * ne);
  for (int64_t t = 0; t < ne; ++t)
    for (int k = 0; k < 4; ++k) Tsoa[k * ne + t] = T[4 * t + k];
  HB_CHECK(m->tets.ensure(sizeof(int32_t) * 4 * ne));
  HB_CHECK(m->geo.ensure(sizeof(double) * geo.size()));
  HB_CHECK(m->dmask.ensure(n_nodes));
  HB_CHECK(m->of.ensure(sizeof(int32_t) * 3 * nof));
  HB_CHECK(m->ofn.ensure(sizeof(double) * 4 * nof));
  HB_CHECK(m->oid.ensure(sizeof(int32_t) * nof));
  std::vector<double> massd(n_nodes, 0.0);
  for (int64_t t = 0; t < ne; ++t)
    for (int k = 0; k < 4; ++k) massd[T[4 * t + k]] += geo[(size_t)hb::GEO_V * ne + t] / 10.0;
  HB_CHECK(m->mass.ensure(sizeof(double) * n_nodes));
  HB_CHECK(hipMemcpy(m->mass.p, massd.data(), sizeof(double) * n_nodes, hipMemcpyHostToDevice));
  HB_CHECK(hipMemcpy(m->tets.p, Tsoa.data(), sizeof(int32_t) * 4 * ne, hipMemcpyHostToDevice));
  HB_CHECK(hipMemcpy(m->geo.p, geo.data(), sizeof(double) * geo.size(), hipMemcpyHostToDevice));
  HB_CHECK(hipMemcpy(m->dmask.p, dmask.data(), n_nodes, hipMemcpyHostToDevice));
  if (nof) {
    HB_CHECK(hipMemcpy(m->of.p, ofv.data(), sizeof(int32_t) * 3 * nof, hipMemcpyHostToDevice));
    HB_CHECK(hipMemcpy(m->ofn.p, ofn.data(), sizeof(double) * 4 * nof, hipMemcpyHostToDevice));
    HB_CHECK(hipMemcpy(m->oid.p, oid.data(), sizeof(int32_t) * nof, hipMemcpyHostToDevice));
  }
  DevMesh& d = m->dm;
  d.n = n_nodes;
  d.ne = ne;
  d.nof = nof;
  d.n_out = n_outlets;
  d.tets = m->tets.as<int32_t>();
  d.geo = m->geo.as<double>();
  d.dmask = m->dmask.as<uint8_t>();
  d.of = m->of.as<int32_t>();
  d.ofn = m->ofn.as<double>();
  d.oid = m->oid.as<int32_t>();
  d.mass = m->mass.as<double>();
  {
    const int sizes[4] = {32, 16, 8, 4};
    for (int i = 0; i < 4; ++i) {
      const int rc = build_blocks(m->bmaps[i], T, ne, sizes[i]);
      if (rc) return rc;
    }
  }
  for (int64_t a = 0; a < n_nodes; ++a) {
    m->n_dirichlet += dmask[a];
    m->n_inlet += inlet[a];
    if (inlet[a] && !wall[a]) m->inlet_nodes.push_back((int32_t)a);
  }
  if (!m->inlet_nodes.empty()) {
    HB_CHECK(m->inlet_dev.ensure(sizeof(int32_t) * m->inlet_nodes.size()));
    HB_CHECK(hipMemcpy(m->inlet_dev.p, m->inlet_nodes.data(),
                       sizeof(int32_t) * m->inlet_nodes.size(), hipMemcpyHostToDevice));
  }
  m->n_reoriented = reoriented;
  m->mean_vol = vsum / ne;
  *out = m.release();
  return HB_OK;
}

void hb_mesh_destroy(hb_mesh* mesh) { delete mesh; }

int hb_set_timing(hb_mesh* m, int32_t enable) {
  if (!m) return fail(HB_ERR_ARG, "NULL mesh");
  if (enable && !m->ev[0])
    for (auto& e : m->ev) HB_CHECK(hipEventCreate(&e));
  m->timing = enable != 0;
  m->timed_call = false;
  return HB_OK;
}

int hb_last_timings(const hb_mesh* mesh, double* ms) {
  if (!mesh || !ms) return fail(HB_ERR_ARG, "NULL argument");
  if (!mesh->timing || !mesh->timed_call) return fail(HB_ERR_ARG, "no timed call");
  HB_CHECK(hipEventSynchronize(mesh->ev[6]));
  for (int k = 0; k < 6; ++k) {
    float t = 0.f;
    HB_CHECK(hipEventElapsedTime(&t, mesh->ev[k], mesh->ev[k + 1]));
    ms[k] = t;
  }
  return HB_OK;
}

int hb_mesh_info(const hb_mesh* m, int64_t* info) {
  if (!m || !info) return fail(HB_ERR_ARG, "NULL argument");
  info[0] = m->dm.n;
  info[1] = m->dm.ne;
  info[2] = m->n_dirichlet;
  info[3] = m->dm.nof;
  info[4] = m->dm.n_out;
  info[5] = m->n_reoriented;
  info[6] = m->n_inlet;
  info[7] = (int64_t)m->bytes_held();
  return HB_OK;
}

int hb_residual(const hb_mesh* mesh, const hb_params* prm, const hb_bc* bc, const double* Y,
                double* R, void* stream) {
  if (!mesh || !Y || !R) return fail(HB_ERR_ARG, "NULL argument");
  hb_mesh* m = const_cast<hb_mesh*>(mesh);
  hipStream_t st = (hipStream_t)stream;
  int rc = prepare(m, prm, bc, st);
  if (rc) return rc;
  Workspace& w = m->ws;
  const int N = w.N;
  const Phys p = make_phys(prm, 0.0);
  Ptrs s = small_ptrs(m);
  const double* tab = w.tab.as<double>();
  HB_CHECK(mark(m, 0, st));
  HB_CHECK(hb::modal_to_samples<double, double>(m->dm, N, Y, bc->dirichlet, 0, tab, w.Sy.as<double>(),
                                w.acc.as<double>(), s.Q, m->dm.n_out * N, st));
  HB_CHECK(mark(m, 1, st));
  HB_CHECK(mark(m, 2, st));
  if (s.R) HB_CHECK(hb::outlet_flux<double>(m->dm, N, w.Sy.as<double>(), s.Q, st));
  HB_CHECK(mark(m, 3, st));
  HB_CHECK(hb::elem_residual(m->dm, p, w.Sy.as<double>(), w.acc.as<double>(),
                             pick_blocks(m, N), st));
  HB_CHECK(mark(m, 4, st));
  HB_CHECK(hb::face_residual(m->dm, p, w.Sy.as<double>(), s.hs, s.R, s.Q, w.acc.as<double>(), st));
  HB_CHECK(mark(m, 5, st));
  HB_CHECK(hb::samples_to_modal<double, double>(m->dm, N, w.acc.as<double>(), 1, 1, hb::NCH, tab, R, st));
  HB_CHECK(mark(m, 6, st));
  return HB_OK;
}

int hb_jvp(const hb_mesh* mesh, const hb_params* prm, const hb_bc* bc, const double* Y,
           const void* V, void* JV, int32_t flags, void* stream) {
  if (!mesh || !Y || !V || !JV) return fail(HB_ERR_ARG, "NULL argument");
  if (flags & ~3) return fail(HB_ERR_ARG, "unknown flags");
  const int kind = flags & 1;
  if ((flags & HB_F32) && kind != HB_JV_EXACT)
    return fail(HB_ERR_ARG, "HB_F32 is available for HB_JV_EXACT only");
  hb_mesh* m = const_cast<hb_mesh*>(mesh);
  hipStream_t st = (hipStream_t)stream;
  int rc = prepare(m, prm, bc, st);
  if (rc) return rc;
  Workspace& w = m->ws;
  const int N = w.N;
  const Phys p = make_phys(prm, 0.0);
  Ptrs s = small_ptrs(m);
  const double* tab = w.tab.as<double>();
  double* Sy = w.Sy.as<double>();
  double* Sv = w.Sv.as<double>();
  double* acc = w.acc.as<double>();
  if (flags & HB_F32) {
    rc = ensure_f32(m);
    if (rc) return rc;
    float* Sy32 = w.Sy32.as<float>();
    float* Sv32 = w.Sv32.as<float>();
    float* acc32 = w.acc32.as<float>();
    HB_CHECK(mark(m, 0, st));
    HB_CHECK(hb::modal_to_samples<double, float>(m->dm, N, Y, bc->dirichlet, 0, tab, Sy32,
                                                 nullptr, nullptr, 0, st));
    HB_CHECK(mark(m, 1, st));
    HB_CHECK(hb::modal_to_samples<float, float>(m->dm, N, (const float*)V, bc->dirichlet, 1, tab,
                                                Sv32, acc32, s.dQ, m->dm.n_out * N, st));
    HB_CHECK(mark(m, 2, st));
    if (s.R) HB_CHECK(hb::outlet_flux<float>(m->dm, N, Sv32, s.dQ, st));
    HB_CHECK(mark(m, 3, st));
    HB_CHECK(hb::elem_jvp_exact<float>(m->dm, p, Sy32, Sv32, acc32,
                                       pick_blocks(m, N), st));
    HB_CHECK(mark(m, 4, st));
    HB_CHECK(hb::face_jvp<float>(m->dm, p, Sy32, Sv32, s.R, s.dQ, acc32, st));
    HB_CHECK(mark(m, 5, st));
    HB_CHECK(hb::samples_to_modal<float, float>(m->dm, N, acc32, 1, 1, hb::NCH, tab, (float*)JV,
                                                st));
    HB_CHECK(mark(m, 6, st));
    return HB_OK;
  }
  HB_CHECK(mark(m, 0, st));
  HB_CHECK(hb::modal_to_samples<double, double>(m->dm, N, Y, bc->dirichlet, 0, tab, Sy, nullptr, nullptr, 0, st));
  HB_CHECK(mark(m, 1, st));
  HB_CHECK(hb::modal_to_samples<double, double>(m->dm, N, (const double*)V, bc->dirichlet, 1, tab, Sv, acc, s.dQ,
                                m->dm.n_out * N, st));
  HB_CHECK(mark(m, 2, st));
  if (kind == HB_JV_EXACT && s.R) HB_CHECK(hb::outlet_flux<double>(m->dm, N, Sv, s.dQ, st));
  HB_CHECK(mark(m, 3, st));
  if (kind == HB_JV_EXACT)
    HB_CHECK(hb::elem_jvp_exact<double>(m->dm, p, Sy, Sv, acc, pick_blocks(m, N), st));
  else
    HB_CHECK(hb::elem_jvp_paper(m->dm, p, Sy, Sv, acc, st));
  HB_CHECK(mark(m, 4, st));
  if (kind == HB_JV_EXACT) HB_CHECK(hb::face_jvp<double>(m->dm, p, Sy, Sv, s.R, s.dQ, acc, st));
  HB_CHECK(mark(m, 5, st));
  HB_CHECK(hb::samples_to_modal<double, double>(m->dm, N, acc, kind == HB_JV_EXACT, 1, hb::NCH, tab, (double*)JV,
                                st));
  HB_CHECK(mark(m, 6, st));
  return HB_OK;
}

// ------------------------------------------------------------ time marching
// One step of the GLS time-marching solver (Section 3, eq. tauhat) at one
// time level: the K = 0 pipeline with the time table's derivative entry
// c1/dt (generalized-alpha, rho_inf = 0: c1 = alpha_m/gamma = 1.5), the
// step history subtracted from the H u channels, no -H N_A test term and
// omega-hat^2 inside tau's bracket.
namespace {
constexpr double kTmC1 = 1.5;

int tm_prepare(hb_mesh* m, const hb_params* prm, const hb_tm_step* tm, hipStream_t st,
               Phys& p) {
  if (!tm) return fail(HB_ERR_ARG, "tm is NULL");
  if (!(tm->dt > 0) || !std::isfinite(tm->dt)) return fail(HB_ERR_ARG, "dt must be positive");
  if (!(tm->omega_hat >= 0) || !std::isfinite(tm->omega_hat))
    return fail(HB_ERR_ARG, "omega_hat must be finite and >= 0");
  if (!tm->y_old || !tm->a_old || !tm->dirichlet)
    return fail(HB_ERR_ARG, "tm.y_old, tm.a_old and tm.dirichlet are required");
  if (!prm) return fail(HB_ERR_ARG, "params is NULL");
  hb_params p0 = *prm;
  p0.K = 0;
  const hb_bc bc0 = {tm->dirichlet, tm->outlet_h, tm->outlet_R};
  int rc = prepare(m, &p0, &bc0, st);
  if (rc) return rc;
  Workspace& w = m->ws;
  std::vector<double> tab(hb::TAB_COUNT, 0.0);
  tab[hb::TAB_BINV] = 1.0;
  tab[hb::TAB_BDER] = kTmC1 / tm->dt;
  tab[hb::TAB_FWD] = 1.0;
  tab[hb::TAB_H] = kTmC1 / tm->dt;
  if (tab != w.tab_host) {
    w.tab_host = tab;
    HB_CHECK(hipMemcpyAsync(w.tab.p, w.tab_host.data(), sizeof(double) * tab.size(),
                            hipMemcpyHostToDevice, st));
  }
  p = make_phys(&p0, 0.0);
  p.tau_add = tm->omega_hat * tm->omega_hat;
  return HB_OK;
}
}  // namespace

int hb_tm_residual(const hb_mesh* mesh, const hb_params* prm, const hb_tm_step* tm,
                   const double* Y, double* R, void* stream) {
  if (!mesh || !Y || !R) return fail(HB_ERR_ARG, "NULL argument");
  hb_mesh* m = const_cast<hb_mesh*>(mesh);
  hipStream_t st = (hipStream_t)stream;
  Phys p;
  int rc = tm_prepare(m, prm, tm, st, p);
  if (rc) return rc;
  Workspace& w = m->ws;
  Ptrs s = small_ptrs(m);
  const double* tab = w.tab.as<double>();
  double* Sy = w.Sy.as<double>();
  double* acc = w.acc.as<double>();
  HB_CHECK(hb::modal_to_samples<double, double>(m->dm, 1, Y, tm->dirichlet, 0, tab, Sy, acc, s.Q,
                                                m->dm.n_out, st));
  HB_CHECK(hb::tm_history(m->dm, Sy, tm->y_old, tm->a_old, kTmC1 / tm->dt, kTmC1 - 1.0, st));
  if (s.R) HB_CHECK(hb::outlet_flux<double>(m->dm, 1, Sy, s.Q, st));
  HB_CHECK(hb::elem_residual(m->dm, p, Sy, acc, pick_blocks(m, 1), st));
  HB_CHECK(hb::face_residual(m->dm, p, Sy, s.hs, s.R, s.Q, acc, st));
  HB_CHECK(hb::samples_to_modal<double, double>(m->dm, 1, acc, 0, 1, hb::NCH, tab, R, st));
  return HB_OK;
}

int hb_tm_jvp(const hb_mesh* mesh, const hb_params* prm, const hb_tm_step* tm, const double* Y,
              const double* V, double* JV, void* stream) {
  if (!mesh || !Y || !V || !JV) return fail(HB_ERR_ARG, "NULL argument");
  hb_mesh* m = const_cast<hb_mesh*>(mesh);
  hipStream_t st = (hipStream_t)stream;
  Phys p;
  int rc = tm_prepare(m, prm, tm, st, p);
  if (rc) return rc;
  Workspace& w = m->ws;
  Ptrs s = small_ptrs(m);
  const double* tab = w.tab.as<double>();
  double* Sy = w.Sy.as<double>();
  double* Sv = w.Sv.as<double>();
  double* acc = w.acc.as<double>();
  HB_CHECK(hb::modal_to_samples<double, double>(m->dm, 1, Y, tm->dirichlet, 0, tab, Sy, nullptr,
                                                nullptr, 0, st));
  HB_CHECK(hb::tm_history(m->dm, Sy, tm->y_old, tm->a_old, kTmC1 / tm->dt, kTmC1 - 1.0, st));
  HB_CHECK(hb::modal_to_samples<double, double>(m->dm, 1, V, tm->dirichlet, 1, tab, Sv, acc, s.dQ,
                                                m->dm.n_out, st));
  if (s.R) HB_CHECK(hb::outlet_flux<double>(m->dm, 1, Sv, s.dQ, st));
  HB_CHECK(hb::elem_jvp_exact<double>(m->dm, p, Sy, Sv, acc, pick_blocks(m, 1), st));
  HB_CHECK(hb::face_jvp<double>(m->dm, p, Sy, Sv, s.R, s.dQ, acc, st));
  HB_CHECK(hb::samples_to_modal<double, double>(m->dm, 1, acc, 0, 1, hb::NCH, tab, JV, st));
  return HB_OK;
}

int hb_jacobi(const hb_mesh* mesh, const hb_params* prm, const hb_bc* bc, const double* Y,
              double shift, double* D, void* stream) {
  if (!mesh || !Y || !D) return fail(HB_ERR_ARG, "NULL argument");
  if (!std::isfinite(shift) || shift < 0) return fail(HB_ERR_ARG, "shift must be finite, >= 0");
  hb_mesh* m = const_cast<hb_mesh*>(mesh);
  hipStream_t st = (hipStream_t)stream;
  int rc = prepare(m, prm, bc, st);
  if (rc) return rc;
  Workspace& w = m->ws;
  const int N = w.N;
  const Phys p = make_phys(prm, shift);
  const double* tab = w.tab.as<double>();
  HB_CHECK(hb::modal_to_samples<double, double>(m->dm, N, Y, bc->dirichlet, 0, tab, w.Sy.as<double>(), nullptr,
                                nullptr, 0, st));
  HB_CHECK(hb::vec_zero<double>(w.dg.as<double>(), m->dm.n * 2 * N, st));
  HB_CHECK(hb::elem_jacobi(m->dm, p, w.Sy.as<double>(), w.dg.as<double>(), 0, st));
  HB_CHECK(hb::jacobi_out(m->dm, N, 2, w.dg.as<double>(), D, nullptr, st));
  return HB_OK;
}

int hb_precond_apply(const hb_mesh* mesh, const hb_params* prm, const hb_bc* bc, const double* Y,
                     double shift, const hb_precond_opts* o, int32_t op, const double* X,
                     double* OUT, void* stream) {
  if (!mesh || !Y || !X || !OUT || !o) return fail(HB_ERR_ARG, "NULL argument");
  if (op != 0 && op != 1) return fail(HB_ERR_ARG, "op must be 0 or 1");
  if (!std::isfinite(shift) || shift < 0) return fail(HB_ERR_ARG, "shift must be finite, >= 0");
  if (o->sweeps < 1 || o->cycles < 1 || !(o->weight > 0 && o->weight <= 1) || o->coarse_max < 1 ||
      o->coarse_max > 256 || (o->aggregation != 0 && o->aggregation != 1) ||
      !(o->coarse_weight > 0 && o->coarse_weight <= 2) || (o->smoother != 0 && o->smoother != 1) ||
      (o->wcycle != 0 && o->wcycle != 1) || (o->fp32 != 0 && o->fp32 != 1))
    return fail(HB_ERR_ARG, "bad preconditioner options");
  hb_mesh* m = const_cast<hb_mesh*>(mesh);
  hipStream_t st = (hipStream_t)stream;
  int rc = prepare(m, prm, bc, st);
  if (rc) return rc;
  Workspace& w = m->ws;
  const int N = w.N;
  rc = ensure_precond(m, o->coarse_max, o->aggregation == 0, N);
  if (rc) return rc;
  const double* tab = w.tab.as<double>();
  const Phys p = make_phys(prm, shift);
  HB_CHECK(hb::modal_to_samples<double, double>(m->dm, N, Y, bc->dirichlet, 0, tab,
                                                w.Sy.as<double>(), nullptr, nullptr, 0, st));
  HB_CHECK(hb::precond_setup(m->pc, m->dm, p, w.Sy.as<double>(), shift, o->sweeps, o->cycles,
                             o->weight, o->coarse_weight, o->smoother, o->wcycle, o->fp32, st));
  // X (Dirichlet velocity entries dropped) to samples [n][7][N]
  HB_CHECK(hb::modal_to_samples<double, double>(m->dm, N, X, bc->dirichlet, 1, tab,
                                                w.Sv.as<double>(), nullptr, nullptr, 0, st));
  if (op == 0) {
    HB_CHECK((hb::precond_matvec<double, double>(m->pc, m->dm.n, w.Sv.as<double>(), hb::NCH,
                                                 m->pcz.as<double>(), st)));
  } else {
    int sing = 0;
    HB_CHECK(hb::precond_singular(m->pc, &sing, st));
    if (sing) return fail(HB_ERR_NOCONV, "singular coarsest-level matrix");
    HB_CHECK((hb::precond_apply<double, double>(m->pc, m->dm.n, w.Sv.as<double>(), hb::NCH,
                                                m->pcz.as<double>(), st)));
  }
  HB_CHECK(hb::samples_to_modal<double, double>(m->dm, N, m->pcz.as<double>(), 0, 1, 4, tab, OUT,
                                                st));
  return HB_OK;
}

int hb_outlet_flow(const hb_mesh* mesh, const hb_params* prm, const hb_bc* bc, const double* Y,
                   double* Q, double* defect, void* stream) {
  if (!mesh || !Y || !Q) return fail(HB_ERR_ARG, "NULL argument");
  hb_mesh* m = const_cast<hb_mesh*>(mesh);
  hipStream_t st = (hipStream_t)stream;
  int rc = prepare(m, prm, bc, st);
  if (rc) return rc;
  Workspace& w = m->ws;
  const int N = w.N;
  const int nout = m->dm.n_out;
  Ptrs s = small_ptrs(m);
  const double* tab = w.tab.as<double>();
  // Q (zeroed by the transform) holds the flux of every outlet at every sample
  HB_CHECK(hb::modal_to_samples<double, double>(m->dm, N, Y, bc->dirichlet, 0, tab,
                                                w.Sy.as<double>(), w.acc.as<double>(), s.Q,
                                                nout * N, st));
  HB_CHECK(hb::outlet_flux<double>(m->dm, N, w.Sy.as<double>(), s.Q, st));
  std::vector<double> qh((size_t)nout * N);
  HB_CHECK(hipMemcpyAsync(qh.data(), s.Q, sizeof(double) * qh.size(), hipMemcpyDeviceToHost, st));
  if (defect) {
    // continuity rows of eq. Rmc summed over all nodes, per sample
    const Phys p = make_phys(prm, 0.0);
    HB_CHECK(hb::elem_residual(m->dm, p, w.Sy.as<double>(), w.acc.as<double>(),
                               pick_blocks(m, N), st));
    HB_CHECK(m->sb.uc.ensure(sizeof(double) * N));
    double* sums = m->sb.uc.as<double>();
    HB_CHECK(hb::channel_sum(w.acc.as<double>(), m->dm.n, hb::NCH, N, 3, sums, st));
    HB_CHECK(hipMemcpyAsync(defect, sums, sizeof(double) * N, hipMemcpyDeviceToHost, st));
  }
  HB_CHECK(hipStreamSynchronize(st));
  std::memcpy(Q, qh.data(), sizeof(double) * qh.size());
  return HB_OK;
}

int hb_precond_levels(const hb_mesh* mesh, int64_t* sizes, int32_t max, int32_t* n_levels) {
  if (!mesh || !n_levels || (max > 0 && !sizes)) return fail(HB_ERR_ARG, "NULL argument");
  *n_levels = hb::precond_levels(mesh->pc, sizes, max);
  return HB_OK;
}

}  // extern "C"

// ------------------------------------------------------------ the solver

namespace {

// Inexact Newton-GMRES in time-sample space.  T is the Krylov type: double
// for the FP64 solve; float for the mixed-precision solve, where the basis
// vectors, the Jacobian-vector products (on an FP32 copy of the state) and
// the GMRES solution are FP32 while the residual, the preconditioner, the
// Gram-Schmidt coefficients (FP64 accumulation) and the Newton update stay
// FP64, so that the outer iteration refines to the FP64 residual.
// workgroup cap of the fused second Gram-Schmidt update and norm
constexpr int kNormBlocks = 4096;

template <typename T>
struct Solver {
  hb_mesh* m;
  const hb_params* prm;
  hipStream_t st;
  int N;
  int64_t L;
  int restart;
  int nblk;
  int jv_kind;
  const double* binv = nullptr;  // per-node time blocks, or NULL for the diagonal
  bool use_pc = false;           // mean-flow modal preconditioner (m->pc)
  bool jv64 = false;  // FP32 basis with FP64 Jacobian-vector products (HB_F32_BASIS)
  bool use_graphs = false;     // replay captured Arnoldi steps
  bool timed_apply = true;     // false while capturing
  const double* shift_dev = nullptr;
  SolverBufs* sb = nullptr;
  // time-marching step (hb_tm_march): tau-hat term, no -H z term, and the
  // step history subtracted from the state's H u channels
  double tau_add = 0.0;
  int use_z = 1;
  const double* hist_y = nullptr;
  const double* hist_a = nullptr;
  double hist_cu = 0.0, hist_ca = 0.0;
  double jv_ms = 0.0;
  double pc_ms = 0.0;
  int n_jv = 0;
  bool jv_pending[2] = {false, false};

  T* Q(int j) { return sb->basis.as<T>() + (size_t)j * L; }
  // the state as seen by the Krylov operator
  const T* state() {
    if constexpr (std::is_same<T, double>::value) return m->ws.Sy.as<double>();
    else return m->ws.Sy32.as<float>();
  }
  T* dir() {
    if constexpr (std::is_same<T, double>::value) return m->ws.Sv.as<double>();
    else return m->ws.Sv32.as<float>();
  }
  T* accum() {
    if constexpr (std::is_same<T, double>::value) return m->ws.acc.as<double>();
    else return m->ws.acc32.as<float>();
  }

  int alloc() {
    sb = &m->sb;
    HB_CHECK(sb->basis.ensure(sizeof(T) * (size_t)(restart + 1) * L));
    HB_CHECK(sb->xvec.ensure(sizeof(T) * L));
    HB_CHECK(sb->rvec.ensure(sizeof(T) * L));
    HB_CHECK(sb->tmp.ensure(sizeof(T) * L));
    HB_CHECK(sb->partial.ensure(sizeof(double) *
                                std::max<size_t>((size_t)(restart + 2) * nblk, kNormBlocks)));
    HB_CHECK(sb->hdev.ensure(sizeof(double) * (4 * (size_t)(restart + 1) + 8)));
    const size_t slot = 2 * (size_t)(restart + 1) + 1;
    if (sb->hpin_n < slot * restart + 1) {  // + one slot for the pseudo-time shift
      if (sb->hpin) HB_CHECK(hipHostFree(sb->hpin));
      sb->hpin = nullptr;
      sb->hpin_n = 0;
      HB_CHECK(hipHostMalloc((void**)&sb->hpin, sizeof(double) * (slot * restart + 1)));
      sb->hpin_n = slot * restart + 1;
    }
    HB_CHECK(sb->shift.ensure(sizeof(double)));
    if (use_graphs && !sb->gstream) HB_CHECK(hipStreamCreateWithFlags(&sb->gstream, hipStreamNonBlocking));
    for (auto& e : sb->evh)
      if (!e) HB_CHECK(hipEventCreate(&e));
    for (auto& e : sb->evj)
      if (!e) HB_CHECK(hipEventCreate(&e));
    if constexpr (!std::is_same<T, double>::value) {
      int rc = ensure_f32(m);
      if (rc) return rc;
    }
    return HB_OK;
  }

  // FP32 copy of the state (mixed precision), after every state change.
  int sync_state() {
    if constexpr (!std::is_same<T, double>::value)
      if (!jv64)
        HB_CHECK(hb::vec_copy_scaled<float, double>(m->ws.Sy32.as<float>(), m->ws.Sy.as<double>(),
                                                  m->dm.n * hb::NCH * N, 1.0, st));
    return HB_OK;
  }

  int residual(double* r, double& nrm) {
    Workspace& w = m->ws;
    Ptrs s = small_ptrs(m);
    const double* tab = w.tab.as<double>();
    Phys p = make_phys(prm, 0.0);
    p.tau_add = tau_add;
    double* Sy = w.Sy.as<double>();
    HB_CHECK(hb::prepare_direction<double, double>(m->dm, N, Sy, hb::NCH, nullptr, nullptr, 0,
                                                   tab, Sy, w.acc.as<double>(), s.Q,
                                                   m->dm.n_out * N, st));
    if (hist_y)
      HB_CHECK(hb::tm_history(m->dm, Sy, hist_y, hist_a, hist_cu, hist_ca, st));
    if (s.R) HB_CHECK(hb::outlet_flux<double>(m->dm, N, Sy, s.Q, st));
    HB_CHECK(hb::elem_residual(m->dm, p, Sy, w.acc.as<double>(), pick_blocks(m, N), st));
    HB_CHECK(hb::face_residual(m->dm, p, Sy, s.hs, s.R, s.Q, w.acc.as<double>(), st));
    HB_CHECK(hb::finish_rows<double, double>(m->dm, N, w.acc.as<double>(), use_z, tab, nullptr,
                                             r, st));
    int rc = sync_state();
    if (rc) return rc;
    return norm<double>(r, nrm);
  }

  template <typename V>
  int norm(const V* x, double& out) {
    HB_CHECK(hb::vec_dots<V>(x, L, 1, x, L, sb->partial.as<double>(), nblk, sb->hdev.as<double>(), st));
    double v = 0.0;
    HB_CHECK(hipMemcpyAsync(&v, sb->hdev.p, sizeof(double), hipMemcpyDeviceToHost, st));
    HB_CHECK(hipStreamSynchronize(st));
    out = std::sqrt(v);
    return HB_OK;
  }

  // w = J M^-1 q (+ shift mass), Dirichlet momentum rows = q.
  int apply(const T* q, T* wout, double shift) {
    Workspace& w = m->ws;
    Ptrs s = small_ptrs(m);
    const double* tab = w.tab.as<double>();
    Phys p = make_phys(prm, shift);
    p.shift_dev = shift_dev;
    p.tau_add = tau_add;
    if constexpr (!std::is_same<T, double>::value) {
      if (jv64) return apply_f64(q, wout, p, s, tab);
    }
    T* Sv = dir();
    T* acc = accum();
    const int pr = n_jv & 1;
    if (timed_apply) {
      int rc = timer_start(pr);
      if (rc) return rc;
    }
    if (use_pc) {
      HB_CHECK((hb::precond_apply<T, double>(m->pc, m->dm.n, q, 4, m->pcz.as<double>(), st)));
      if (timed_apply) {
        int rc = timer_mid(pr);
        if (rc) return rc;
      }
      HB_CHECK((hb::prepare_direction<double, T>(m->dm, N, m->pcz.as<double>(), 4, nullptr,
                                                 nullptr, 1, tab, Sv, acc, s.dQ,
                                                 m->dm.n_out * N, st)));
    } else {
      if (timed_apply) {
        int rc = timer_mid(pr);
        if (rc) return rc;
      }
      HB_CHECK(hb::prepare_direction<T, T>(m->dm, N, q, 4, w.dinv.as<double>(), binv, 1, tab,
                                           Sv, acc, s.dQ, m->dm.n_out * N, st));
    }
    if (jv_kind == HB_JV_EXACT) {
      if (s.R) HB_CHECK(hb::outlet_flux<T>(m->dm, N, Sv, s.dQ, st));
      HB_CHECK(hb::elem_jvp_exact<T>(m->dm, p, state(), Sv, acc, pick_blocks(m, N),
                                     st));
      HB_CHECK(hb::face_jvp<T>(m->dm, p, state(), Sv, s.R, s.dQ, acc, st));
      HB_CHECK(hb::finish_rows<T, T>(m->dm, N, acc, use_z, tab, q, wout, st));
    } else {
      if constexpr (std::is_same<T, double>::value) {
        HB_CHECK(hb::elem_jvp_paper(m->dm, p, w.Sy.as<double>(), Sv, acc, st));
        HB_CHECK(hb::finish_rows<double, double>(m->dm, N, acc, 0, tab, q, wout, st));
      } else {
        return fail(HB_ERR_ARG, "the paper tangent is available in FP64 only");
      }
    }
    return timed_apply ? timer_stop(pr) : HB_OK;
  }

  // Jv timing with two event pairs used in turn; a pair's previous
  // duration is collected (waited for) before the pair is reused.
  int timer_start(int pr) {
    if (jv_pending[pr]) {
      int rc = collect_jv(pr);
      if (rc) return rc;
    }
    HB_CHECK(hipEventRecord(sb->evj[3 * pr], st));
    return HB_OK;
  }
  // between the preconditioner and the Jacobian-vector product
  int timer_mid(int pr) {
    HB_CHECK(hipEventRecord(sb->evj[3 * pr + 1], st));
    return HB_OK;
  }
  int timer_stop(int pr) {
    HB_CHECK(hipEventRecord(sb->evj[3 * pr + 2], st));
    jv_pending[pr] = true;
    ++n_jv;
    return HB_OK;
  }

  // FP32 basis vector in, FP64 Jacobian-vector product on the FP64 state,
  // FP32 basis vector out.
  int apply_f64(const T* q, T* wout, const Phys& p, const Ptrs& s, const double* tab) {
    Workspace& w = m->ws;
    double* Sv = w.Sv.as<double>();
    double* acc = w.acc.as<double>();
    const int pr = n_jv & 1;
    if (timed_apply) {
      int rc = timer_start(pr);
      if (rc) return rc;
    }
    if (use_pc) {
      HB_CHECK((hb::precond_apply<T, double>(m->pc, m->dm.n, q, 4, m->pcz.as<double>(), st)));
      if (timed_apply) {
        int rc = timer_mid(pr);
        if (rc) return rc;
      }
      HB_CHECK((hb::prepare_direction<double, double>(m->dm, N, m->pcz.as<double>(), 4, nullptr,
                                                      nullptr, 1, tab, Sv, acc, s.dQ,
                                                      m->dm.n_out * N, st)));
    } else {
      if (timed_apply) {
        int rc = timer_mid(pr);
        if (rc) return rc;
      }
      HB_CHECK((hb::prepare_direction<T, double>(m->dm, N, q, 4, w.dinv.as<double>(), binv, 1,
                                                  tab, Sv, acc, s.dQ, m->dm.n_out * N, st)));
    }
    if (s.R) HB_CHECK(hb::outlet_flux<double>(m->dm, N, Sv, s.dQ, st));
    HB_CHECK(hb::elem_jvp_exact<double>(m->dm, p, w.Sy.as<double>(), Sv, acc,
                                        pick_blocks(m, N), st));
    HB_CHECK(hb::face_jvp<double>(m->dm, p, w.Sy.as<double>(), Sv, s.R, s.dQ, acc, st));
    HB_CHECK((hb::finish_rows<double, T>(m->dm, N, acc, use_z, tab, q, wout, st)));
    return timed_apply ? timer_stop(pr) : HB_OK;
  }

  // Everything a captured Arnoldi step depends on by value: sizes, device
  // pointers and the fluid parameters baked into its kernel arguments.
  std::vector<uintptr_t> graph_key() {
    Workspace& w = m->ws;
    const Ptrs s = small_ptrs(m);
    auto bits = [](double v) {
      uint64_t u;
      std::memcpy(&u, &v, sizeof(u));
      return (uintptr_t)u;
    };
    return {(uintptr_t)N, (uintptr_t)restart, (uintptr_t)L, (uintptr_t)nblk,
            (uintptr_t)jv_kind, (uintptr_t)jv64, (uintptr_t)sizeof(T),
            (uintptr_t)sb->basis.p, (uintptr_t)sb->partial.p, (uintptr_t)sb->hdev.p,
            (uintptr_t)sb->shift.p, (uintptr_t)binv, (uintptr_t)w.dinv.p, (uintptr_t)w.tab.p,
            (uintptr_t)w.small.p, (uintptr_t)s.R, (uintptr_t)w.Sy.p, (uintptr_t)w.Sv.p,
            (uintptr_t)w.acc.p, (uintptr_t)w.Sy32.p, (uintptr_t)w.Sv32.p, (uintptr_t)w.acc32.p,
            (uintptr_t)pick_blocks(m, N).ptr, (uintptr_t)use_pc, (uintptr_t)m->pc,
            (uintptr_t)m->pcz.p, bits(prm->rho), bits(prm->mu), bits(prm->period),
            bits(prm->C_I), bits(prm->beta_bf)};
  }

  // Adds the duration of a recorded Jv (waits for it).
  int collect_jv(int pr) {
    HB_CHECK(hipEventSynchronize(sb->evj[3 * pr + 2]));
    float ms = 0.f, mp = 0.f;
    HB_CHECK(hipEventElapsedTime(&mp, sb->evj[3 * pr], sb->evj[3 * pr + 1]));
    HB_CHECK(hipEventElapsedTime(&ms, sb->evj[3 * pr + 1], sb->evj[3 * pr + 2]));
    jv_ms += ms;
    pc_ms += mp;
    jv_pending[pr] = false;
    return HB_OK;
  }
  int collect_all_jv() {
    for (int pr = 0; pr < 2; ++pr)
      if (jv_pending[pr]) {
        int rc = collect_jv(pr);
        if (rc) return rc;
      }
    return HB_OK;
  }

  // Right-preconditioned restarted GMRES on (J M^-1) x = -r; CGS2.
  //
  // The Arnoldi steps run on the device without host round trips: the
  // Gram-Schmidt coefficients stay on the device, the new basis vector is
  // normalised there, and the coefficients are copied to pinned host slots.
  // The host reads step j's coefficients (Givens rotations, convergence
  // test) while step j+1 is already queued, so the GPU never waits for the
  // host; a converged cycle has computed one step more than it uses.
  int gmres(const double* r, double shift, double eta, int max_it, int& iters) {
    T* x = sb->xvec.as<T>();
    T* rl = sb->rvec.as<T>();
    HB_CHECK(hb::vec_zero<T>(x, L, st));
    HB_CHECK((hb::vec_copy_scaled<T, double>(rl, r, L, -1.0, st)));
    double beta;
    int rc = norm<T>(rl, beta);
    if (rc) return rc;
    iters = 0;
    if (beta == 0.0) return HB_OK;
    const double target = eta * beta;
    const int mr = restart;
    const size_t slot = 2 * (size_t)(mr + 1) + 1;
    std::vector<double> Hm((size_t)(mr + 1) * mr), cs(mr), sn(mr), g(mr + 1), yv(mr);
    double bc = beta;
    double* h1 = sb->hdev.as<double>();
    double* h2 = h1 + (mr + 1);
    double* h3 = h2 + (mr + 1);
    double* ydev = h1 + slot;
    if (use_graphs) {
      // the shift is read from device memory, so captured steps stay valid
      sb->hpin[slot * mr] = shift;
      HB_CHECK(hipMemcpyAsync(sb->shift.p, sb->hpin + slot * mr, sizeof(double),
                              hipMemcpyHostToDevice, st));
      shift_dev = sb->shift.as<double>();
      const std::vector<uintptr_t> key = graph_key();
      if (key != sb->gkey) {
        sb->drop_graphs();
        sb->gkey = key;
      }
      if ((int)sb->gexec.size() < mr) sb->gexec.resize(mr, nullptr);
    }
    // kernels of Arnoldi step j: w = A v_j, two Gram-Schmidt passes, |w|^2,
    // normalisation (no host work in between, so the sequence can be captured)
    auto step_kernels = [&](int j) -> int {
      T* wj = Q(j + 1);
      int rc2 = apply(Q(j), wj, shift);
      if (rc2) return rc2;
      double* part = sb->partial.as<double>();
      HB_CHECK(hb::vec_mdots<T>(Q(0), L, j + 1, wj, L, part, nblk, h1, st));
      HB_CHECK(hb::vec_axpy_multi<T>(wj, Q(0), L, j + 1, h1, -1.0, L, st));
      HB_CHECK(hb::vec_mdots<T>(Q(0), L, j + 1, wj, L, part, nblk, h2, st));
      HB_CHECK(hb::vec_axpy_norm<T>(wj, Q(0), L, j + 1, h2, L, part, kNormBlocks, h3, st));
      HB_CHECK(hb::vec_scale_inv_norm<T>(wj, L, h3, st));
      return HB_OK;
    };
    // capture step j on the private stream (nothing runs during capture)
    auto capture = [&](int j) -> int {
      hipStream_t saved = st;
      st = sb->gstream;
      timed_apply = false;
      hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
      const int rc2 = e == hipSuccess ? step_kernels(j) : HB_OK;
      hipGraph_t g = nullptr;
      const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(st, &g) : e;
      st = saved;
      timed_apply = true;
      if (rc2 != HB_OK || e2 != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        if (rc2 != HB_OK) return rc2;
        return fail(HB_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e2));
      }
      const hipError_t e3 = hipGraphInstantiate(&sb->gexec[j], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e3 != hipSuccess) {
        sb->gexec[j] = nullptr;
        return fail(HB_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e3));
      }
      return HB_OK;
    };
    // queue Arnoldi step j and the copy of its coefficients to the host
    auto enqueue = [&](int j) -> int {
      if (use_graphs) {
        if (!sb->gexec[j]) {
          const int rc2 = capture(j);
          if (rc2) return rc2;
        }
        const int pr = n_jv & 1;
        int rc2 = timer_start(pr);
        if (rc2) return rc2;
        rc2 = timer_mid(pr);
        if (rc2) return rc2;
        HB_CHECK(hipGraphLaunch(sb->gexec[j], st));
        rc2 = timer_stop(pr);
        if (rc2) return rc2;
      } else {
        const int rc2 = step_kernels(j);
        if (rc2) return rc2;
      }
      HB_CHECK(hipMemcpyAsync(sb->hpin + (size_t)j * slot, h1, sizeof(double) * slot,
                              hipMemcpyDeviceToHost, st));
      HB_CHECK(hipEventRecord(sb->evh[j & 1], st));
      return HB_OK;
    };
    while (true) {
      HB_CHECK((hb::vec_copy_scaled<T, T>(Q(0), rl, L, 1.0 / bc, st)));
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = bc;
      int jend = 0;
      bool done = false;
      // host side of step j: Hessenberg column, Givens rotation, test
      auto finish = [&](int j) -> int {
        HB_CHECK(hipEventSynchronize(sb->evh[j & 1]));
        const double* hh = sb->hpin + (size_t)j * slot;
        double* col = &Hm[(size_t)j * (mr + 1)];
        for (int k = 0; k <= j; ++k) col[k] = hh[k] + hh[(mr + 1) + k];
        const double hn = std::sqrt(std::max(hh[2 * (mr + 1)], 0.0));
        if (!std::isfinite(hn)) return fail(HB_ERR_NAN, "non-finite Krylov vector");
        col[j + 1] = hn;
        for (int k = 0; k < j; ++k) {
          const double a = col[k], b = col[k + 1];
          col[k] = cs[k] * a + sn[k] * b;
          col[k + 1] = -sn[k] * a + cs[k] * b;
        }
        const double den = std::hypot(col[j], col[j + 1]);
        cs[j] = den > 0 ? col[j] / den : 1.0;
        sn[j] = den > 0 ? col[j + 1] / den : 0.0;
        col[j] = den;
        col[j + 1] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        ++iters;
        jend = j + 1;
        if (std::fabs(g[j + 1]) <= target || iters >= max_it || hn == 0.0) done = true;
        return HB_OK;
      };
      for (int j = 0; j < mr && !done; ++j) {
        if (iters + j - jend < max_it) {  // queue step j unless the budget is spent
          rc = enqueue(j);
          if (rc) return rc;
        }
        if (j > 0) {
          rc = finish(j - 1);
          if (rc) return rc;
        }
        if (!done && j == mr - 1) {
          rc = finish(j);
          if (rc) return rc;
        }
      }
      for (int i = jend - 1; i >= 0; --i) {
        double v = g[i];
        for (int k = i + 1; k < jend; ++k) v -= Hm[(size_t)k * (mr + 1) + i] * yv[k];
        const double d = Hm[(size_t)i * (mr + 1) + i];
        yv[i] = d != 0.0 ? v / d : 0.0;
      }
      HB_CHECK(hipMemcpyAsync(ydev, yv.data(), sizeof(double) * jend, hipMemcpyHostToDevice, st));
      HB_CHECK(hb::vec_axpy_multi<T>(x, Q(0), L, jend, ydev, 1.0, L, st));
      HB_CHECK(hipStreamSynchronize(st));
      if (done && (std::fabs(g[jend]) <= target || iters >= max_it)) break;
      // restart: rl = -r - (J M^-1) x
      rc = apply(x, sb->tmp.as<T>(), shift);
      if (rc) return rc;
      HB_CHECK((hb::vec_copy_scaled<T, double>(rl, r, L, -1.0, st)));
      double one = 1.0;
      HB_CHECK(hipMemcpyAsync(ydev, &one, sizeof(double), hipMemcpyHostToDevice, st));
      HB_CHECK(hb::vec_axpy_multi<T>(rl, sb->tmp.as<T>(), L, 1, ydev, -1.0, L, st));
      rc = norm<T>(rl, bc);
      if (rc) return rc;
      if (bc <= target || iters >= max_it) break;
    }
    return collect_all_jv();
  }

  // state += M^-1 x (FP64), skipping Dirichlet velocity entries.
  int update_state() {
    Workspace& w = m->ws;
    const double* tab = w.tab.as<double>();
    if (use_pc) {
      HB_CHECK((hb::precond_apply<T, double>(m->pc, m->dm.n, sb->xvec.as<T>(), 4,
                                             m->pcz.as<double>(), st)));
      HB_CHECK(hb::vec_mul_dinv_add<double>(w.Sy.as<double>(), m->pcz.as<double>(), nullptr,
                                            m->dm.dmask, m->dm.n, N, hb::NCH, 4, 1.0, st));
    } else if (binv) {
      HB_CHECK((hb::prepare_direction<T, double>(m->dm, N, sb->xvec.as<T>(), 4, w.dinv.as<double>(),
                                                 binv, 1, tab, w.Sv.as<double>(), nullptr,
                                                 nullptr, 0, st)));
      HB_CHECK(hb::vec_mul_dinv_add<double>(w.Sy.as<double>(), w.Sv.as<double>(), nullptr,
                                            m->dm.dmask, m->dm.n, N, hb::NCH, hb::NCH, 1.0, st));
    } else {
      HB_CHECK(hb::vec_mul_dinv_add<T>(w.Sy.as<double>(), sb->xvec.as<T>(), w.dinv.as<double>(),
                                       m->dm.dmask, m->dm.n, N, hb::NCH, 4, 1.0, st));
    }
    return HB_OK;
  }
};

template <typename T>
int newton_run(hb_mesh* m, const hb_params* prm, const hb_bc* bc, double* Y,
               const hb_solve_opts* opts, hb_solve_report* report, hipStream_t st,
               std::chrono::steady_clock::time_point t0) {
  Solver<T> S;
  S.m = m;
  S.prm = prm;
  S.st = st;
  S.N = m->ws.N;
  S.L = m->dm.n * 4 * S.N;
  S.restart = opts->restart;
  S.nblk = 1024;  // workgroups per vector slice of the Krylov reductions (upper bound)
  S.jv_kind = opts->jv_kind == HB_JV_PAPER ? HB_JV_PAPER : HB_JV_EXACT;
  S.jv64 = opts->precision == HB_F32_BASIS;
  // on request, launch-bound sizes replay captured Arnoldi steps (not with
  // the mean-flow multigrid: its cycles take the pseudo-time coefficient by
  // value, which a captured step would keep from the step it was captured in)
  S.use_graphs = opts->graphs == 1 && S.L <= ((int64_t)1 << 22) && S.jv_kind == HB_JV_EXACT &&
                 opts->precond != HB_PREC_MEANFLOW;
  const int N = S.N;
  const int64_t L = S.L;
  int rc = S.alloc();
  if (rc) return rc;
  if (opts->precond == HB_PREC_NODE_TIME) {
    if (N > 64) return fail(HB_ERR_ARG, "HB_PREC_NODE_TIME needs K <= 31");
    HB_CHECK(m->ws.binv.ensure(sizeof(double) * (size_t)m->dm.n * N * N));
    S.binv = m->ws.binv.as<double>();
  } else if (opts->precond == HB_PREC_MEANFLOW) {
    rc = ensure_precond(m, kCoarseMax, opts->amg_aggregation == 0, N);
    if (rc) return rc;
    S.use_pc = true;
  } else if (opts->precond != HB_PREC_JACOBI) {
    return fail(HB_ERR_ARG, "unknown preconditioner");
  }
  const int amg_nu = opts->amg_sweeps > 0 ? opts->amg_sweeps : 2;
  const int amg_cyc = opts->amg_cycles > 0 ? opts->amg_cycles : 1;
  const double amg_w = opts->amg_weight > 0 ? opts->amg_weight : 0.7;
  const double amg_g = opts->amg_coarse_weight > 0 ? opts->amg_coarse_weight : 0.7;
  Workspace& w = m->ws;
  const double* tab = w.tab.as<double>();
  HB_CHECK(hb::modal_to_samples<double, double>(m->dm, N, Y, bc->dirichlet, 0, tab,
                                                w.Sy.as<double>(), nullptr, nullptr, 0, st));

  // initial pseudo step: dt = cfl h_c / u_c (Section 2.3)
  const double hc = std::cbrt(6.0 * std::sqrt(2.0) * m->mean_vol);
  double uc = 0.0;
  if (!m->inlet_nodes.empty()) {
    HB_CHECK(m->sb.uc.ensure(sizeof(double) * N));
    HB_CHECK(hb::inlet_speed(bc->dirichlet, m->dm.n, N, m->inlet_dev.as<int32_t>(),
                             (int64_t)m->inlet_nodes.size(), tab, m->sb.uc.as<double>(), st));
    std::vector<double> us(N);
    HB_CHECK(hipMemcpyAsync(us.data(), m->sb.uc.p, sizeof(double) * N, hipMemcpyDeviceToHost,
                            st));
    HB_CHECK(hipStreamSynchronize(st));
    for (double v : us) uc = std::max(uc, v);
  }
  const double dt0 = uc > 0 ? opts->cfl * hc / uc : opts->cfl * hc;
  const double dt_max = opts->cfl_max > 0 ? dt0 * opts->cfl_max / opts->cfl : 1e6 * dt0;

  HB_CHECK(m->sb.rbuf.ensure(sizeof(double) * L));
  double* r = m->sb.rbuf.as<double>();
  double rn = 0.0;
  rc = S.residual(r, rn);
  if (rc) return rc;
  report->r0 = rn;
  if (!std::isfinite(rn)) return fail(HB_ERR_NAN, "non-finite initial residual");
  const double ref = opts->r_ref > 0 ? opts->r_ref : rn;
  report->r_ref = ref;
  const double ser_ref = std::max(ref, rn);
  // Pseudo-step control.  The first step follows switched evolution
  // relaxation from max(reference, initial residual), so a start whose
  // residual is already below the reference takes a larger step at once;
  // later steps scale dt by the residual ratio of the accepted step (at
  // least by dt_growth when the residual did not grow).  A pseudo-time step
  // is not a descent step (the mass shift holds the velocity back while the
  // pressure follows the continuity rows at once), so ordinary growth of the
  // residual is accepted; only a step whose residual exceeds reject_ratio
  // times the previous one (or is not finite) is damped, y + alpha delta
  // with alpha = 1/2, 1/4, ... 1/64, until the residual falls below the
  // previous one, keeping the trial with the smallest residual; the next
  // pseudo step is scaled by sqrt(alpha), never below 1/100 of the first.
  const double reject = opts->reject_ratio == 0 ? 100.0 : opts->reject_ratio;
  const double grow_min = opts->dt_growth > 0 ? opts->dt_growth : 1.0;
  constexpr int kMaxHalve = 6;
  double dt = std::min(dt0 * ser_ref / std::max(rn, 1e-300), dt_max);
  const double dt_min = 0.01 * dt0;
  const int64_t sy_len = m->dm.n * hb::NCH * N;
  const size_t sy_bytes = sizeof(double) * (size_t)sy_len;
  if (reject > 0) {
    HB_CHECK(m->sb.sysave.ensure(sy_bytes));
    HB_CHECK(m->sb.syfull.ensure(sy_bytes));
  }
  // forcing term: fixed, or the Eisenstat-Walker choice eta_k =
  // 0.9 (|r_k| / |r_k-1|)^2, kept above 0.9 eta_k-1^2 when that exceeds 0.1,
  // within [gmres_eta / 10, max(gmres_eta, 0.5)], and never asking more of
  // the linear solve than the Newton target (eta |r_k| >= rtol r_ref / 2)
  double eta = opts->gmres_eta;
  const double eta_lo = 0.1 * opts->gmres_eta, eta_hi = std::max(opts->gmres_eta, 0.5);
  int status = HB_ERR_NOCONV;
  int it = 0;
  for (;; ++it) {
    if (rn <= opts->rtol * ref) {
      status = HB_OK;
      break;
    }
    if (it >= opts->max_newton) break;
    if (opts->forcing == 1)
      eta = std::min(eta_hi, std::max(eta, 0.5 * opts->rtol * ref / std::max(rn, 1e-300)));
    const double shift = opts->c1 * prm->rho / dt;
    const Phys pj = make_phys(prm, shift);
    if (S.use_pc) {
      HB_CHECK(hb::precond_setup(m->pc, m->dm, pj, w.Sy.as<double>(), shift, amg_nu, amg_cyc,
                                 amg_w, amg_g, opts->amg_smoother, opts->amg_wcycle,
                                 opts->amg_fp32, st));
    } else {
      const int nc = S.binv ? 4 : 2;
      HB_CHECK(hb::vec_zero<double>(w.dg.as<double>(), m->dm.n * nc * N, st));
      HB_CHECK(hb::elem_jacobi(m->dm, pj, w.Sy.as<double>(), w.dg.as<double>(), S.binv ? 1 : 0,
                               st));
      HB_CHECK(hb::jacobi_out(m->dm, N, nc, w.dg.as<double>(), nullptr, w.dinv.as<double>(), st));
      if (S.binv)
        HB_CHECK(hb::block_factor(m->dm, N, w.dg.as<double>(), m->dm.mass, prm->rho, tab,
                                  w.binv.as<double>(), st));
    }
    int gi = 0;
    rc = S.gmres(r, shift, eta, opts->max_gmres, gi);
    if (rc) return rc;
    report->gmres_iters += gi;
    double* Sy = w.Sy.as<double>();
    double* save = m->sb.sysave.as<double>();
    double* full = m->sb.syfull.as<double>();
    if (reject > 0) HB_CHECK(hipMemcpyAsync(save, Sy, sy_bytes, hipMemcpyDeviceToDevice, st));
    rc = S.update_state();
    if (rc) return rc;
    double rn_new = 0.0;
    rc = S.residual(r, rn_new);
    if (rc) return rc;
    double alpha = 1.0;
    if (reject > 0 && !(rn_new <= reject * rn)) {
      // damped steps along the same direction; keep the best one
      HB_CHECK(hipMemcpyAsync(full, Sy, sy_bytes, hipMemcpyDeviceToDevice, st));
      double best = std::isfinite(rn_new) ? rn_new : HUGE_VAL, best_a = 1.0, a = 1.0;
      for (int h = 0; h < kMaxHalve; ++h) {
        a *= 0.5;
        HB_CHECK(hb::vec_blend(Sy, save, full, sy_len, a, st));
        double ra = 0.0;
        rc = S.residual(r, ra);
        if (rc) return rc;
        if (std::isfinite(ra) && ra < best) {
          best = ra;
          best_a = a;
        }
        if (ra <= rn) break;
      }
      ++report->rejected;
      if (best_a != a) {  // the last trial is not the best: restore the best
        HB_CHECK(hb::vec_blend(Sy, save, full, sy_len, best_a, st));
        rc = S.residual(r, rn_new);
        if (rc) return rc;
      } else {
        rn_new = best;
      }
      alpha = best_a;
    }
    if (!std::isfinite(rn_new)) {
      report->newton_iters = it + 1;
      return fail(HB_ERR_NAN, "non-finite residual");
    }
    if (opts->verbose)
      std::fprintf(stderr, "hb newton %d: |r| = %.3e  gmres %d  dt %.3e  alpha %.3g\n", it + 1,
                   rn_new, gi, dt, alpha);
    if (alpha < 1.0) {
      dt = std::max(dt * std::sqrt(alpha), dt_min);
    } else {
      double f = rn / std::max(rn_new, 1e-300);
      if (rn_new <= rn) f = std::max(f, grow_min);
      dt = std::min(dt * std::max(f, 0.1), dt_max);
    }
    if (opts->forcing == 1) {
      const double ratio = rn_new / std::max(rn, 1e-300);
      double e = 0.9 * ratio * ratio;
      const double keep = 0.9 * eta * eta;
      if (keep > 0.1) e = std::max(e, keep);
      eta = std::min(eta_hi, std::max(eta_lo, e));
    }
    rn = rn_new;
  }
  report->newton_iters = it;
  report->r_final = rn;
  {
    // mass balance at the final state: the continuity rows summed over all
    // nodes equal the net boundary outflow (sum_A N_A = 1), relative to the
    // largest total outlet flow over the samples
    Ptrs s = small_ptrs(m);
    const int nout = m->dm.n_out;
    HB_CHECK(hb::vec_zero<double>(s.Q, (int64_t)nout * N, st));
    HB_CHECK(hb::outlet_flux<double>(m->dm, N, w.Sy.as<double>(), s.Q, st));
    HB_CHECK(m->sb.uc.ensure(sizeof(double) * N));
    HB_CHECK(hb::channel_sum(r, m->dm.n, 4, N, 3, m->sb.uc.as<double>(), st));
    std::vector<double> qh((size_t)nout * N), dh(N);
    HB_CHECK(hipMemcpyAsync(qh.data(), s.Q, sizeof(double) * qh.size(), hipMemcpyDeviceToHost,
                            st));
    HB_CHECK(hipMemcpyAsync(dh.data(), m->sb.uc.p, sizeof(double) * N, hipMemcpyDeviceToHost, st));
    HB_CHECK(hipStreamSynchronize(st));
    double qmax = 0.0, dmax = 0.0;
    for (int k = 0; k < N; ++k) {
      double q = 0.0;
      for (int o = 0; o < nout; ++o) q += qh[(size_t)o * N + k];
      qmax = std::max(qmax, std::fabs(q));
      dmax = std::max(dmax, std::fabs(dh[k]));
    }
    report->mass_defect = qmax > 0 ? dmax / qmax : dmax;
  }
  HB_CHECK(hb::samples_to_modal<double, double>(m->dm, N, w.Sy.as<double>(), 0, 0, hb::NCH, tab,
                                                Y, st));
  HB_CHECK(hipStreamSynchronize(st));
  report->status = status;
  report->jv_ms = S.jv_ms;
  report->pc_ms = S.pc_ms;
  report->n_jv = S.n_jv;
  report->wall_s =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (status != HB_OK) return fail(status, "Newton iteration limit reached");
  return HB_OK;
}

// Time marching of the GLS comparison solver: n_steps generalized-alpha
// steps, each solved by Newton-GMRES on the step residual with its exact
// Jacobian (right-preconditioned by the Jacobi diagonal of the paper's
// tangent plus c1 rho/dt times the mass diagonal).
int tm_march_run(hb_mesh* m, const hb_params* prm, const hb_bc* bc, double* Y, double* A,
                 double* traj, const hb_tm_opts* o, hb_tm_report* rep, hipStream_t st,
                 std::chrono::steady_clock::time_point t0) {
  const int64_t n = m->dm.n;
  const int nout = m->dm.n_out;
  const int Nb = 2 * prm->K + 1;
  const double omega = 6.283185307179586476925286766559 / prm->period;
  const double dt = o->dt;
  HB_CHECK(m->tm_yold.ensure(sizeof(double) * 4 * n));
  HB_CHECK(m->tm_g.ensure(sizeof(double) * 3 * n));
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024));
  HB_CHECK(m->tm_part.ensure(sizeof(double) * (2 * (size_t)nb + 2)));
  double* yold = m->tm_yold.as<double>();
  double* g = m->tm_g.as<double>();
  double* part = m->tm_part.as<double>();
  double* sums = part + 2 * nb;
  hb_params p0 = *prm;
  p0.K = 0;
  std::vector<double> hstep(nout > 0 ? nout : 1, 0.0);
  Solver<double> S;
  S.m = m;
  S.prm = &p0;
  S.st = st;
  S.N = 1;
  S.L = 4 * n;
  S.restart = o->restart;
  S.nblk = 1024;
  S.jv_kind = HB_JV_EXACT;
  S.use_z = 0;
  bool allocated = false;
  int status = HB_OK;
  for (int k = 0; k < o->n_steps; ++k) {
    const double t1 = o->t0 + (double)(k + 1) * dt;
    double what = o->omega_hat;
    if (what < 0) {  // eq. tauhat from the step's starting state
      HB_CHECK(hb::tm_norms(m->dm, Y, A, part, nb, sums, st));
      double hs2[2] = {0.0, 0.0};
      HB_CHECK(hipMemcpyAsync(hs2, sums, sizeof(hs2), hipMemcpyDeviceToHost, st));
      HB_CHECK(hipStreamSynchronize(st));
      what = hs2[0] > 0 ? std::sqrt(hs2[1] / hs2[0]) : 0.0;
    }
    HB_CHECK(hb::modal_eval(m->dm, prm->K, omega, t1, bc->dirichlet, g, st));
    if (bc->outlet_h)
      for (int q = 0; q < nout; ++q) {
        const double* hq = bc->outlet_h + (size_t)q * Nb;
        double v = hq[0];
        for (int j = 1; j <= prm->K; ++j)
          v += std::cos(j * omega * t1) * hq[2 * j - 1] + std::sin(j * omega * t1) * hq[2 * j];
        hstep[q] = v;
      }
    HB_CHECK(hipMemcpyAsync(yold, Y, sizeof(double) * 4 * n, hipMemcpyDeviceToDevice, st));
    const hb_tm_step tm = {dt, what, yold, A, g, bc->outlet_h ? hstep.data() : nullptr,
                           bc->outlet_R};
    Phys pp;
    int rc = tm_prepare(m, prm, &tm, st, pp);
    if (rc) return rc;
    if (!allocated) {
      rc = S.alloc();
      if (rc) return rc;
      HB_CHECK(m->sb.rbuf.ensure(sizeof(double) * S.L));
      if (o->precond == HB_PREC_MEANFLOW) {
        rc = ensure_precond(m, kCoarseMax, 1, 1);
        if (rc) return rc;
        S.use_pc = true;
      }
      allocated = true;
    }
    S.tau_add = pp.tau_add;
    S.hist_y = yold;
    S.hist_a = A;
    S.hist_cu = kTmC1 / dt;
    S.hist_ca = kTmC1 - 1.0;
    Workspace& w = m->ws;
    const double* tab = w.tab.as<double>();
    HB_CHECK(hb::modal_to_samples<double, double>(m->dm, 1, Y, g, 0, tab, w.Sy.as<double>(),
                                                  nullptr, nullptr, 0, st));
    double* r = m->sb.rbuf.as<double>();
    double rn = 0.0;
    rc = S.residual(r, rn);
    if (rc) return rc;
    if (!std::isfinite(rn)) return fail(HB_ERR_NAN, "non-finite step residual");
    const double target = std::max(o->atol, o->rtol * rn);
    int it = 0;
    while (rn > target && it < o->max_newton) {
      Phys pj = make_phys(&p0, prm->rho * kTmC1 / dt);
      pj.tau_add = pp.tau_add;
      if (S.use_pc) {
        HB_CHECK(hb::precond_setup(m->pc, m->dm, pj, w.Sy.as<double>(), pj.shift, 2, 1, 0.7, 0.7,
                                   0, 0, 0, st));
      } else {
        HB_CHECK(hb::vec_zero<double>(w.dg.as<double>(), n * 2, st));
        HB_CHECK(hb::elem_jacobi(m->dm, pj, w.Sy.as<double>(), w.dg.as<double>(), 0, st));
        HB_CHECK(hb::jacobi_out(m->dm, 1, 2, w.dg.as<double>(), nullptr, w.dinv.as<double>(),
                                st));
      }
      int gi = 0;
      rc = S.gmres(r, 0.0, o->gmres_eta, o->max_gmres, gi);
      if (rc) return rc;
      rep->gmres_iters += gi;
      rc = S.update_state();
      if (rc) return rc;
      rc = S.residual(r, rn);
      if (rc) return rc;
      if (!std::isfinite(rn)) return fail(HB_ERR_NAN, "non-finite step residual");
      ++it;
    }
    rep->newton_iters += it;
    rep->max_step_residual = std::max(rep->max_step_residual, rn);
    if (rn > target) status = HB_ERR_NOCONV;
    HB_CHECK(hb::samples_to_modal<double, double>(m->dm, 1, w.Sy.as<double>(), 0, 0, hb::NCH, tab,
                                                  Y, st));
    HB_CHECK(hb::tm_accel(m->dm, Y, yold, A, 1.0 / dt, st));
    if (traj)
      HB_CHECK(hipMemcpyAsync(traj + (size_t)k * 4 * n, Y, sizeof(double) * 4 * n,
                              hipMemcpyDeviceToDevice, st));
    rep->steps = k + 1;
    if (o->verbose)
      std::fprintf(stderr, "hb tm step %d: t %.4f newton %d |r| %.3e omega_hat %.3e\n", k + 1, t1,
                   it, rn, what);
  }
  HB_CHECK(hipStreamSynchronize(st));
  rep->status = status;
  rep->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (status != HB_OK) return fail(status, "a step reached its Newton iteration limit");
  return HB_OK;
}

}  // namespace

extern "C" {

int hb_tm_march(const hb_mesh* mesh, const hb_params* prm, const hb_bc* bc, double* Y, double* A,
                double* traj, const hb_tm_opts* opts, hb_tm_report* report, void* stream) {
  if (!mesh || !prm || !bc || !Y || !A || !opts || !report) return fail(HB_ERR_ARG, "NULL argument");
  const auto t0 = std::chrono::steady_clock::now();
  std::memset(report, 0, sizeof(*report));
  report->status = HB_ERR_NOCONV;
  int rc = check_params(prm);
  if (rc) return rc;
  if (!bc->dirichlet) return fail(HB_ERR_ARG, "bc.dirichlet is NULL");
  if (!(opts->dt > 0) || !std::isfinite(opts->dt) || !std::isfinite(opts->t0))
    return fail(HB_ERR_ARG, "dt must be positive and t0 finite");
  if (opts->n_steps < 0) return fail(HB_ERR_ARG, "n_steps must be >= 0");
  if (!(opts->rtol > 0) || !(opts->atol >= 0) || !(opts->gmres_eta > 0))
    return fail(HB_ERR_ARG, "rtol and gmres_eta must be positive, atol >= 0");
  if (opts->restart < 1 || opts->restart > 512) return fail(HB_ERR_ARG, "restart must be 1..512");
  if (opts->max_newton < 0 || opts->max_gmres < 1) return fail(HB_ERR_ARG, "bad iteration limits");
  if (std::isnan(opts->omega_hat)) return fail(HB_ERR_ARG, "omega_hat is NaN");
  if (opts->precond != HB_PREC_JACOBI && opts->precond != HB_PREC_MEANFLOW)
    return fail(HB_ERR_ARG, "precond must be HB_PREC_JACOBI or HB_PREC_MEANFLOW");
  return tm_march_run(const_cast<hb_mesh*>(mesh), prm, bc, Y, A, traj, opts, report,
                      (hipStream_t)stream, t0);
}

int hb_newton_solve(const hb_mesh* mesh, const hb_params* prm, const hb_bc* bc, double* Y,
                    const hb_solve_opts* opts, hb_solve_report* report, void* stream) {
  if (!mesh || !Y || !opts || !report) return fail(HB_ERR_ARG, "NULL argument");
  const auto t0 = std::chrono::steady_clock::now();
  std::memset(report, 0, sizeof(*report));
  report->status = HB_ERR_NOCONV;
  if (opts->precision != HB_F64 && opts->precision != HB_MIXED && opts->precision != HB_F32_BASIS)
    return fail(HB_ERR_ARG, "precision must be HB_F64, HB_MIXED or HB_F32_BASIS");
  if (opts->precision != HB_F64 && opts->jv_kind == HB_JV_PAPER)
    return fail(HB_ERR_ARG, "the mixed-precision solve uses the exact Jacobian");
  if (opts->restart < 1 || opts->restart > 512) return fail(HB_ERR_ARG, "restart must be 1..512");
  if (opts->max_newton < 0 || opts->max_gmres < 1) return fail(HB_ERR_ARG, "bad iteration limits");
  if (!(opts->rtol > 0) || !(opts->gmres_eta > 0) || !(opts->cfl > 0) || !(opts->c1 >= 0))
    return fail(HB_ERR_ARG, "rtol, gmres_eta, cfl must be positive");
  if (!std::isfinite(opts->reject_ratio) || !(opts->dt_growth >= 0) ||
      !std::isfinite(opts->dt_growth) || (opts->reject_ratio > 0 && opts->reject_ratio < 1))
    return fail(HB_ERR_ARG, "reject_ratio must be finite (0, < 0 or >= 1), dt_growth >= 0");
  if (opts->amg_sweeps < 0 || opts->amg_cycles < 0 || !(opts->amg_weight >= 0) ||
      opts->amg_weight > 1 || (opts->amg_aggregation != 0 && opts->amg_aggregation != 1) ||
      !(opts->amg_coarse_weight >= 0) || opts->amg_coarse_weight > 2 ||
      (opts->amg_smoother != 0 && opts->amg_smoother != 1) ||
      (opts->amg_wcycle != 0 && opts->amg_wcycle != 1) ||
      (opts->amg_fp32 != 0 && opts->amg_fp32 != 1))
    return fail(HB_ERR_ARG, "bad multigrid options");
  if (opts->forcing != 0 && opts->forcing != 1) return fail(HB_ERR_ARG, "forcing must be 0 or 1");
  hb_mesh* m = const_cast<hb_mesh*>(mesh);
  hipStream_t st = (hipStream_t)stream;
  int rc = prepare(m, prm, bc, st);
  if (rc) return rc;
  if (opts->precision != HB_F64) return newton_run<float>(m, prm, bc, Y, opts, report, st, t0);
  return newton_run<double>(m, prm, bc, Y, opts, report, st, t0);
}

}  // extern "C"
