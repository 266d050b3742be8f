/*
 * hb.h - C interface of the MI355X harmonic-balance (HB) GLS Navier-Stokes
 * library: residual, Jacobian-vector product and Newton-GMRES solve of the
 * time-periodic incompressible Navier-Stokes equations on P1-P1 tetrahedra.
 *
 * The method is that of Jia & Esmaily, "Introducing a harmonic balance
 * Navier-Stokes finite element solver to accelerate cardiovascular
 * simulations" (arXiv 2411.14315):
 *   - problem statement: Section 2.1, eq. NS-time (rigid walls, Dirichlet
 *     data g on inlets and walls, normal traction h on outlets);
 *   - harmonic balance form: Section 2.1, eqs. upghdft and NS-harm
 *     (N = 2K+1 time samples, H = E^-1 Omega E);
 *   - GLS weak form and tau: Section 2.2, eqs. NS-weak and tau;
 *   - discrete residual: Section 2.3, eq. Rmc; backflow stabilisation
 *     (beta = 0.2) on outlets, Section 2.3;
 *   - Newton-Raphson with pseudo time stepping and Jacobi-preconditioned
 *     GMRES: Section 2.3, eqs. NR, splitK, ptangent, K_mat, ctangent.
 *
 * Conventions shared by every call
 * --------------------------------
 * Modal layout.  A nodal field set Y is an array of doubles
 *     Y[f][m][a],  f in {u1, u2, u3, p},  m in 0..2K,  a = node (contiguous)
 * with harmonic order [a_0, a_1, b_1, ..., a_K, b_K], meaning that at time t
 *     q(t) = a_0 + sum_{m=1..K} a_m cos(m w t) + b_m sin(m w t),  w = 2 pi/T.
 * The paper's complex coefficient is q*_m = (a_m - i b_m)/2.  Time samples are
 * t_n = n T / N, n = 0..N-1.  Residual and Jacobian-vector outputs use the
 * same layout and hold the real DFT of the time-sample rows of eq. Rmc:
 *     R[f][0][a] = (1/N) sum_n r_n,  R[f][2m-1][a] = (2/N) sum_n r_n cos(2 pi m n/N),
 *     R[f][2m][a] = (2/N) sum_n r_n sin(2 pi m n/N).
 *
 * Dirichlet nodes are the nodes of wall and inlet faces.  Y's velocity entries
 * there are ignored on input and replaced by the boundary data; the momentum
 * rows of R and JV there are zero; V's velocity entries there are taken as 0.
 * Continuity rows exist at every node (eq. Rmc).
 *
 * Memory.  Arrays documented "device" are caller-owned device allocations
 * (for example torch tensors) on the current HIP device; "host" arrays are
 * read during the call only.  The library owns what hb_mesh_create
 * allocates.  A handle must not be used by two calls at the same time;
 * calls on one handle are ordered by their stream.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = default
 * stream).  hb_residual, hb_jvp and hb_jacobi are asynchronous on it;
 * hb_newton_solve returns after its work has finished.
 *
 * Errors.  Every call returns HB_OK (0) or a negative status; nothing throws
 * across the interface.  hb_last_error() returns a thread-local message for
 * the last failure on the calling thread.
 */
#ifndef HB_H
#define HB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HB_OK = 0,
  HB_ERR_ARG = -1,     /* invalid argument, size or pointer                  */
  HB_ERR_MESH = -2,    /* index out of range, degenerate tetrahedron, bad face */
  HB_ERR_DEVICE = -3,  /* HIP runtime or kernel launch failure               */
  HB_ERR_NOCONV = -4,  /* Newton iteration limit reached before tolerance     */
  HB_ERR_NAN = -5,     /* non-finite residual                                  */
  HB_ERR_OOM = -6      /* device allocation failed                            */
};

/* Boundary group kinds (hb_mesh_create group_kind). */
enum { HB_WALL = 0, HB_INLET = 1, HB_OUTLET = 2 };

/* hb_jvp flags: tangent kind (bit 0) and vector precision (bit 1). */
enum {
  HB_JV_EXACT = 0, /* exact directional derivative of the residual            */
  HB_JV_PAPER = 1, /* the paper's tangent C + P (eqs. ptangent, K_mat, ctangent):
                      frozen advection and tau, stabilisation time terms
                      dropped, no outlet terms                               */
  HB_F64 = 0,
  HB_F32 = 2       /* V and JV are float arrays (mixed-precision path)         */
};

typedef struct hb_mesh hb_mesh;

/* Fluid and discretisation parameters (Section 2.1-2.3). */
typedef struct {
  double rho;     /* density > 0                                  */
  double mu;      /* dynamic viscosity > 0                        */
  double period;  /* cycle duration T > 0; w = 2 pi / T            */
  int32_t K;      /* retained harmonics, 0 <= K <= 32; N = 2K+1    */
  double C_I;     /* tau constant (3 for tetrahedra, eq. tau)      */
  double beta_bf; /* backflow coefficient (0.2 in the paper)       */
} hb_params;

/* Boundary data. */
typedef struct {
  const double* dirichlet; /* device [3][N][n] modal velocity data; only
                              Dirichlet nodes are read (walls: zero)        */
  const double* outlet_h;  /* host [n_outlets][N] modal normal traction h
                              (h = -p_out for a pressure outlet), or NULL
                              for zero traction                              */
  const double* outlet_R;  /* host [n_outlets] resistances, or NULL.  With a
                              resistance the traction is
                              h_n = h_given,n - R Q_n,  Q_n = outlet flux at
                              sample n (a time-local extension; the paper
                              leaves resistance outlets to future work)       */
} hb_bc;

/* Create a mesh handle on the current HIP device.
 *   xyz        host [n_nodes][3] coordinates
 *   tets       host [n_tets][4] 0-based node indices; negatively oriented
 *              tetrahedra are re-oriented by swapping local nodes 2 and 3
 *   faces      host [n_faces][3] boundary triangles (any orientation)
 *   face_group host [n_faces] group index in 0..n_groups-1
 *   group_kind host [n_groups] HB_WALL / HB_INLET / HB_OUTLET
 * Outlet groups are numbered in increasing group index.  Fails with
 * HB_ERR_MESH for out-of-range indices, |V| < 1e-14 * mean|V|, or a face that
 * is not a face of any tetrahedron; HB_ERR_ARG without any outlet group
 * (the pressure would be undetermined).  *out receives the handle. */
int hb_mesh_create(int64_t n_nodes, const double* xyz, int64_t n_tets, const int32_t* tets,
                   int64_t n_faces, const int32_t* faces, const int32_t* face_group,
                   int32_t n_groups, const int32_t* group_kind, hb_mesh** out);

void hb_mesh_destroy(hb_mesh* mesh);

/* info[0..7] = n_nodes, n_tets, n_dirichlet_nodes, n_outlet_faces,
 * n_outlets, n_reoriented, n_inlet_nodes, device bytes held. */
int hb_mesh_info(const hb_mesh* mesh, int64_t* info);

/* R = modal HB residual of eq. Rmc at Y (device [4][N][n] in, out). */
int hb_residual(const hb_mesh* mesh, const hb_params* prm, const hb_bc* bc, const double* Y,
                double* R, void* stream);

/* JV = dR/dY [V] at Y (device arrays; V and JV double, or float with HB_F32).
 * Flags: HB_JV_EXACT or HB_JV_PAPER, optionally | HB_F32. */
int hb_jvp(const hb_mesh* mesh, const hb_params* prm, const hb_bc* bc, const double* Y,
           const void* V, void* JV, int32_t flags, void* stream);

/* Jacobi diagonal of the paper's tangent (Section 2.3: diag(P), since C has
 * a zero diagonal) plus shift * int N_A^2 on the velocity rows, at Y, in time
 * samples: D device [2][N][n], D[0] = velocity rows (equal for the three
 * components; 1 at Dirichlet nodes), D[1] = continuity rows. */
int hb_jacobi(const hb_mesh* mesh, const hb_params* prm, const hb_bc* bc, const double* Y,
              double shift, double* D, void* stream);

/* One step of the GLS time-marching solver that Section 3 compares the HB
 * solver with, at one time level (the K = 0 layout: arrays [f][n]).  The
 * step solves r(u_{n+1}, p_{n+1}) = 0 with the Galerkin/least-squares terms
 * of eq. Rmc, the acceleration a = (c1/dt)(u_{n+1} - u_n) + (1 - c1) a_n of
 * the generalized-alpha method with rho_inf = 0 (c1 = 1.5, the c1 of
 * Section 2.3) in place of H u, no time derivative on the test functions,
 * and tau-hat of eq. tauhat: omega_hat^2 is added inside tau's bracket.
 * prm->K and prm->period are not used.  All device arrays are caller-owned;
 * y_old and a_old must not alias Y, R, V or JV. */
typedef struct {
  double dt;               /* time step > 0                                   */
  double omega_hat;        /* ||du/dt|| / ||u|| of eq. tauhat, >= 0, held
                              fixed over the step                             */
  const double* y_old;     /* device [4][n] state at t_n (velocity rows read) */
  const double* a_old;     /* device [3][n] acceleration at t_n               */
  const double* dirichlet; /* device [3][n] Dirichlet velocity at t_{n+1}     */
  const double* outlet_h;  /* host [n_outlets] traction at t_{n+1}, or NULL   */
  const double* outlet_R;  /* host [n_outlets] resistance, or NULL            */
} hb_tm_step;

/* R = step residual at Y = (u_{n+1}, p_{n+1}) (device [4][n] in, [4][n]
 * out; Y's Dirichlet velocity entries are replaced by tm->dirichlet;
 * momentum rows at Dirichlet nodes are 0).  Asynchronous on the stream.
 * HB_ERR_ARG for dt <= 0, a negative or non-finite omega_hat or a NULL
 * required pointer. */
int hb_tm_residual(const hb_mesh* mesh, const hb_params* prm, const hb_tm_step* tm,
                   const double* Y, double* R, void* stream);

/* JV = exact derivative of hb_tm_residual at Y along V (device [4][n];
 * V's Dirichlet velocity entries are treated as 0).  Asynchronous. */
int hb_tm_jvp(const hb_mesh* mesh, const hb_params* prm, const hb_tm_step* tm, const double* Y,
              const double* V, double* JV, void* stream);

/* Options and report of hb_tm_march. */
typedef struct {
  double t0;          /* time of the initial state                          */
  double dt;          /* time step > 0                                      */
  int32_t n_steps;    /* steps to take, >= 0                                */
  double rtol, atol;  /* a step converges when ||r|| <= max(atol, rtol ||r_0||)
                         (2-norm of the step residual, r_0 at the previous
                         state with the new boundary data)                  */
  double gmres_eta;   /* GMRES relative tolerance per Newton iteration      */
  int32_t restart, max_newton, max_gmres;
  double omega_hat;   /* < 0: omega-hat of eq. tauhat from each step's
                         starting state (mass-weighted velocity norms);
                         >= 0: held at this value                           */
  int32_t verbose;    /* 1: one line per step on stderr                     */
  int32_t precond;    /* HB_PREC_JACOBI (0) or HB_PREC_MEANFLOW (the same
                         multigrid as hb_newton_solve's, K = 0, with the
                         step's 1.5 rho/dt mass term)                        */
} hb_tm_opts;

typedef struct {
  int32_t steps, newton_iters, gmres_iters, status;
  double max_step_residual, wall_s;
} hb_tm_report;

/* March the GLS comparison solver of Section 3 (the step of hb_tm_residual)
 * over n_steps steps t0 + k dt with the boundary data of bc evaluated at
 * each t_{k+1}: modal Dirichlet data (device [3][2K+1][n], prm->K and
 * prm->period give the harmonics) and modal outlet traction (host).  Each
 * step is solved by Newton-GMRES with the exact step Jacobian, right-
 * preconditioned by the Jacobi diagonal of the paper's tangent plus
 * 1.5 rho/dt times the mass diagonal, or by the multigrid of
 * HB_PREC_MEANFLOW (opts->precond).  Y (device [4][n]) and A (device
 * [3][n]) hold the state and acceleration at t0 on entry and at the last
 * step on return; traj (device [n_steps][4][n], or NULL) receives the
 * state after every step.  Synchronous on return.  HB_ERR_NOCONV if a step
 * reached max_newton (the march still completes), HB_ERR_NAN on a
 * non-finite residual, HB_ERR_ARG for invalid options. */
int hb_tm_march(const hb_mesh* mesh, const hb_params* prm, const hb_bc* bc, double* Y, double* A,
                double* traj, const hb_tm_opts* opts, hb_tm_report* report, void* stream);

/* Preconditioners for hb_newton_solve.  HB_PREC_JACOBI is the paper's Jacobi
 * preconditioner diag(P) (Section 2.3).  HB_PREC_NODE_TIME keeps, for every
 * node, the full N x N time block of the exact Jacobian's velocity diagonal:
 * diag_n(K_AA) + rho int N_A^2 H plus the stabilisation's time terms
 * diag(X) H - H diag(X) - rho H diag(T) H with T = int tau N_A^2 and
 * X = int rho tau (u.grad N_A) N_A, inverted exactly per node; the pressure
 * rows keep 1 / L_AA (requires K <= 31).  HB_PREC_MEANFLOW couples space:
 * the tangent with frozen advection and tau (eq. K_mat's P, the Galerkin
 * time term C of eq. ctangent and the stabilisation's time terms), with
 * every coefficient replaced by its mean over the samples, is block-diagonal
 * in the Fourier modes; each mode's complex system (H -> i m w) is
 * approximated by V-cycles of an aggregation multigrid on the node graph
 * (see hb_precond_apply).  All change iteration counts, not the root. */
enum { HB_PREC_JACOBI = 0, HB_PREC_NODE_TIME = 1, HB_PREC_MEANFLOW = 2 };

/* hb_solve_opts.precision: HB_F64 (= 0), or HB_MIXED: FP32 Krylov basis and
 * FP32 Jacobian-vector products (on an FP32 copy of the state) inside GMRES,
 * with the FP64 residual, FP64 Gram-Schmidt coefficients and FP64 Newton
 * update as the outer (iterative refinement) loop; or HB_F32_BASIS: FP32
 * Krylov basis with FP64 Jacobian-vector products (the basis vectors are
 * widened on entry to the operator and rounded on exit), same outer loop.
 * Both reduced-precision forms require HB_JV_EXACT. */
enum { HB_MIXED = 1, HB_F32_BASIS = 2 };

typedef struct {
  double rtol;       /* stop when ||r||_2 <= rtol * r_ref (default 1e-8)              */
  double r_ref;      /* reference norm; <= 0 means ||r(Y_in)||_2                     */
  double gmres_eta;  /* relative linear tolerance (0.03 in the paper)                 */
  double cfl;        /* pseudo step dt = cfl (h_c / u_c) max(r_ref, ||r_0||) / ||r||
                        (Section 2.3 sets dt ~ h_c / u_c; the growth as the
                        residual falls is an addition: switched evolution
                        relaxation)                                               */
  double c1;         /* pseudo-time constant (1.5 for rho_inf = 0)                    */
  int32_t restart;   /* GMRES restart length (default 50)                             */
  int32_t max_newton;
  int32_t max_gmres; /* per Newton step                                               */
  int32_t precision; /* HB_F64, HB_MIXED or HB_F32_BASIS                            */
  int32_t jv_kind;   /* HB_JV_EXACT or HB_JV_PAPER for the Krylov operator            */
  int32_t verbose;   /* print one line per Newton step to stderr                      */
  int32_t precond;   /* HB_PREC_JACOBI (the paper's diag(P)) or HB_PREC_NODE_TIME    */
  double cfl_max;    /* cap of the pseudo step growth, dt <= cfl_max h_c / u_c
                        (<= 0: no cap beyond 1e6 times the initial step)        */
  int32_t graphs;    /* 0: launch the kernels one by one; 1: when 4 N n <= 2^22,
                        the Jv is HB_JV_EXACT and the preconditioner is not
                        HB_PREC_MEANFLOW, capture every Arnoldi step once as a
                        HIP graph (kept with the mesh) and replay it (else the
                        kernels are launched one by one).  Results agree to
                        rounding.  With graphs, report.jv_ms also includes
                        the Gram-Schmidt work of each step.                   */
  int32_t amg_sweeps; /* HB_PREC_MEANFLOW: Jacobi sweeps before and after each
                         coarse correction (0: 2)                               */
  int32_t amg_cycles; /* HB_PREC_MEANFLOW: V-cycles per application (0: 1)      */
  double amg_weight;  /* HB_PREC_MEANFLOW: Jacobi damping (0: 0.7)              */
  double reject_ratio; /* a step whose residual exceeds reject_ratio times the
                          previous one (or is not finite) is damped by 1/2,
                          1/4, ... 1/64 until the residual falls below the
                          previous one; the trial with the smallest residual
                          is kept; 0: 100; < 0: take every full step          */
  double dt_growth;   /* after an accepted step the pseudo step is scaled by the
                         residual ratio, and by at least dt_growth when the
                         residual did not grow (0: 1, plain switched evolution
                         relaxation)                                             */
  int32_t amg_aggregation; /* HB_PREC_MEANFLOW: 0 two passes of pairwise matching,
                              1 a node with its free neighbours                 */
  double amg_coarse_weight; /* HB_PREC_MEANFLOW: weight of the coarse-level
                               correction (0: 0.7)                              */
  int32_t amg_smoother; /* HB_PREC_MEANFLOW: 0 damped block Jacobi, 1 symmetric
                           block Gauss-Seidel over colour classes              */
  int32_t amg_wcycle;   /* HB_PREC_MEANFLOW: 0 V-cycles, 1 W-cycles            */
  int32_t amg_fp32;     /* HB_PREC_MEANFLOW: 0 FP64 cycles; 1 smoothing, residuals
                           and transfers on FP32 vectors and coefficients (the
                           coefficients are assembled in FP64 and rounded; the
                           coarsest-level inverse stays FP64)                  */
  int32_t forcing;      /* GMRES forcing term: 0 gmres_eta at every step; 1 the
                           Eisenstat-Walker choice 0.9 (|r_k| / |r_k-1|)^2
                           (safeguarded by 0.9 eta_k-1^2 when that exceeds
                           0.1), within [gmres_eta / 10, max(gmres_eta, 0.5)]
                           and no tighter than the Newton target needs;
                           the first step uses gmres_eta                      */
} hb_solve_opts;

typedef struct {
  int32_t newton_iters;
  int32_t gmres_iters;
  int32_t status;
  double r0;       /* ||r(Y_in)||_2, time-sample 2-norm  */
  double r_final;
  double r_ref;
  double wall_s;
  double jv_ms;    /* total time spent in the Jacobian-vector products of the
                      Krylov operator (transforms, element and face
                      kernels, scatter; with graphs also Gram-Schmidt) */
  int32_t n_jv;
  int32_t rejected; /* Newton steps taken damped (alpha < 1)          */
  double pc_ms;    /* total time in preconditioner applications inside the
                      Krylov operator (not part of jv_ms)             */
  double mass_defect; /* at the returned state: max over samples of
                         |sum_A r^c_A(t_n)| (the net boundary outflow, since
                         sum_A N_A = 1) over max over samples of the total
                         outlet flow |sum_k Q_k(t_n)|                     */
} hb_solve_report;

/* Inexact Newton with pseudo-time continuation (Section 2.3): the tangent
 * receives c1 rho/dt int N_A N_B on velocity rows, dt grows by switched
 * evolution relaxation (steps that raise the residual beyond reject_ratio
 * are damped); right-preconditioned restarted
 * GMRES with classical Gram-Schmidt run twice.  Y (device [4][N][n]) holds the initial
 * guess on entry and the solution on return.  Returns HB_OK on convergence,
 * HB_ERR_NOCONV with Y = last iterate otherwise; the report is filled in both
 * cases.  The Krylov basis ((restart + 1) x 4 N n values) and the other solver
 * buffers are allocated on first use and kept with the mesh for later calls
 * (counted in hb_mesh_info's device bytes); calls on one mesh must not
 * overlap. */
int hb_newton_solve(const hb_mesh* mesh, const hb_params* prm, const hb_bc* bc, double* Y,
                    const hb_solve_opts* opts, hb_solve_report* report, void* stream);

/* The mean-flow modal preconditioner (HB_PREC_MEANFLOW) on its own, for
 * checking it.  At the state Y (device [4][N][n], Dirichlet entries from bc)
 * and pseudo-time mass coefficient `shift` (>= 0, the c1 rho / dt of the
 * solve), the operator A is, for each harmonic m (H -> i m w), the sample
 * mean of the tangent with frozen advection and tau: eq. K_mat's blocks,
 * the Galerkin time term of eq. ctangent and the stabilisation's time
 * terms, without outlet terms; Dirichlet velocity rows and columns removed.
 * op = 0: OUT = A X.  op = 1: OUT = M^-1 X, M^-1 = `cycles` V-cycles of an
 * aggregation multigrid with `sweeps` block-Jacobi sweeps (weight `weight`)
 * before and after each coarse correction (weight `coarse_weight`)
 * per level and a dense inverse on the coarsest level, which holds at most
 * `coarse_max` nodes (a mesh with at most coarse_max nodes is solved
 * exactly).  X and OUT are device [4][N][n] modal arrays; X's Dirichlet
 * velocity entries are taken as 0 and OUT's are 0.  The hierarchy is built
 * on first use and kept with the mesh.  Asynchronous on the stream.
 * HB_ERR_ARG for a bad op, sizes or options; HB_ERR_NOCONV if the
 * coarsest-level matrix is singular (op = 1 only; waits for the stream). */
typedef struct {
  int32_t sweeps;        /* >= 1                                              */
  int32_t cycles;        /* >= 1                                              */
  double weight;         /* Jacobi damping, (0, 1]                            */
  int32_t coarse_max;    /* 1..256                                            */
  int32_t aggregation;   /* 0 pairwise matching twice, 1 node + neighbours    */
  double coarse_weight;  /* weight of the coarse-level correction, (0, 2]     */
  int32_t smoother;      /* 0 damped block Jacobi, 1 symmetric block Gauss-
                            Seidel over colour classes (weight unused)        */
  int32_t wcycle;        /* 0 V-cycle, 1 W-cycle                              */
  int32_t fp32;          /* 0 FP64 cycles, 1 FP32 cycles (as amg_fp32)        */
} hb_precond_opts;
int hb_precond_apply(const hb_mesh* mesh, const hb_params* prm, const hb_bc* bc, const double* Y,
                     double shift, const hb_precond_opts* opts, int32_t op, const double* X,
                     double* OUT, void* stream);
/* Outlet flow rates and mass balance at Y (device [4][N][n]; Dirichlet entries
 * from bc): Q (host [n_outlets][N]) = int_{outlet k} u(t_n) . n, the flux
 * through each outlet group at each sample time (exact for P1 fields); defect
 * (host [N], or NULL) = sum over all nodes of the continuity rows of eq. Rmc
 * at each sample, which equals the net outflow through the whole boundary
 * (sum_A N_A = 1, so the stabilisation part cancels): Q_out - Q_in.  For a
 * converged solution it vanishes with the residual.  Waits for the stream. */
int hb_outlet_flow(const hb_mesh* mesh, const hb_params* prm, const hb_bc* bc, const double* Y,
                   double* Q, double* defect, void* stream);

/* Node counts of the preconditioner's levels (finest first): sizes[0..max-1];
 * *n_levels = number of levels (0 before the hierarchy is built). */
int hb_precond_levels(const hb_mesh* mesh, int64_t* sizes, int32_t max, int32_t* n_levels);
/* The mean-flow multigrid's hierarchy of a mesh's node graph, built on the
 * host alone (no device work; for checking it): tets (host [ne][4], 0-based,
 * indices < n), aggregation 0 (two passes of pairwise matching) or 1 (a node
 * with its free neighbours), coarsening until at most coarse_max (1..256)
 * nodes remain or a level no longer shrinks by 10 %.  sizes (host
 * [max_levels]) receives the node counts of the first max_levels levels,
 * *n_levels the number of levels; agg0 (host [n] or NULL) the aggregate of
 * each node of the finest level (-1 when there is one level); colour0 (host
 * [n] or NULL) the colour class of each finest-level node (no two
 * neighbours share one; the Gauss-Seidel smoother's classes).  HB_ERR_ARG
 * for bad sizes, options or indices. */
int hb_precond_hierarchy(int64_t n, int64_t ne, const int32_t* tets, int32_t coarse_max,
                         int32_t aggregation, int32_t max_levels, int64_t* sizes,
                         int32_t* n_levels, int32_t* agg0, int32_t* colour0);

/* Per-stage timing of hb_residual / hb_jvp for profiling.  When enabled,
 * those calls record HIP events on their stream between stages:
 *   0 state to samples, 1 direction to samples, 2 outlet flux,
 *   3 element kernel, 4 outlet faces, 5 samples to modal rows.
 * hb_last_timings waits for the last call's events and writes the stage
 * durations in milliseconds to ms[0..5] (0 for stages a call does not
 * run).  Returns HB_ERR_ARG if timing was not enabled for the last call. */
int hb_set_timing(hb_mesh* mesh, int32_t enable);
int hb_last_timings(const hb_mesh* mesh, double* ms);

/* ------------------------------------------------------------------------
 * Learned Newton warm start (a data-driven initial guess, outside the paper's
 * method: the paper notes HB solutions as a source of training data for
 * machine-learning models, Section 4).  A multilayer perceptron with BF16
 * weights and FP32 accumulation maps problem parameters to POD coefficients
 * of the modal solution; hb_pod_expand forms the guess.  The final FP64
 * residual of hb_newton_solve decides: callers keep the plain start when the
 * guess's residual is larger.
 *
 * Parameter layout: for each layer l, W_l [out_l][in_l] row-major then
 * b_l [out_l], as FP32 values (held internally as BF16 plus an FP32 Adam
 * master copy).  Hidden layers use ReLU, the last is linear.  Loss: mean
 * squared error (1/(B out)) sum (y - t)^2.  Device arrays are caller-owned;
 * calls are asynchronous on `stream` except where a host result is returned.
 * A network handle must not be used by two calls at the same time. */
typedef struct hb_mlp hb_mlp;

/* widths[0..n_layers]: input width, hidden widths, output width.  params
 * (host, n_params floats) or NULL for a seeded He-uniform initialisation. */
int hb_mlp_create(int32_t n_layers, const int32_t* widths, const float* params, uint64_t seed,
                  hb_mlp** out);
void hb_mlp_destroy(hb_mlp* net);
int hb_mlp_num_params(const hb_mlp* net, int64_t* count);
/* The current (BF16-rounded) parameters as floats, host [n_params]. */
int hb_mlp_get_params(const hb_mlp* net, float* host_out);
/* Y (device [B][out]) = net(X) (device [B][in]). */
int hb_mlp_forward(hb_mlp* net, const float* X, int32_t B, float* Y, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * forward pass as hb_mlp_forward, Y (device [B][out]) = net(X) (device
 * [B][in]), with the hidden activations in a fixed library-owned device array
 * of 16 MiB per GPU (held until the process ends) instead of the handle's
 * buffers.  Requires B * (largest hidden or output width) <= 1,048,576, else
 * HB_ERR_ARG.  Calls no allocating routine.  Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU race (order them on one stream).
 * Asynchronous on the stream. */
int hb_mlp_forward_noalloc(const hb_mlp* net, const float* X, int32_t B, float* Y, void* stream);
/* Mean squared error against T (device [B][out]) and its gradient with
 * respect to the parameters: grad device [n_params] (NULL = internal
 * buffer used by hb_mlp_adam_step); *loss (host, may be NULL) waits for the
 * result. */
int hb_mlp_loss_grad(hb_mlp* net, const float* X, const float* T, int32_t B, float* grad,
                     double* loss, void* stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected) with the given
 * gradient (device, or NULL for the internal one). */
int hb_mlp_adam_step(hb_mlp* net, const float* grad, float lr, void* stream);
/* Y[i] = base[i] + mean[i] + sum_k coef[k] basis[k][i], i < L (device
 * arrays; base [L] double or NULL for none, basis [r][L] double, coef [r]
 * float; r = 0 allows basis and coef NULL).  Y may alias base.  A model
 * trained on corrections to the plain start passes that start as base. */
int hb_pod_expand(int64_t L, int32_t r, const double* base, const double* mean,
                  const double* basis, const float* coef, double* Y, void* stream);

/* Proper orthogonal decomposition of a snapshot set by the method of
 * snapshots, for the network's targets.  Snapshot i is row i of S minus row
 * i of B (device [ns][L] FP64 row-major; B NULL for none; both read only).
 * With c_i = snapshot i - mean and the Gram matrix G_ij = c_i . c_j =
 * sum_k V_ik lam_k V_jk (lam descending), the modes are
 * basis_k = sum_i V_ik c_i / sqrt(lam_k) (orthonormal) for k < r, where r
 * counts the leading lam_k > max(0, floor_rel lam_0) among the first r_max.
 * Outputs: mean (device [L]); basis (device [r_max][L], rows >= r left as
 * they are); coef (host [ns][r_max]) = V_ik sqrt(lam_k) = c_i . basis_k,
 * zero for k >= r; lam (host [ns]) every eigenvalue of G, descending;
 * *r_out = r.  Mean, Gram matrix (FP64 atomics, so not bitwise
 * reproducible) and modes run on the device; the ns x ns eigenproblem on
 * the host (hb_sym_eig).  Needs 1 <= ns <= 4096, 1 <= r_max <= ns; device
 * scratch of ns (ns + r) doubles is allocated per call.  Waits for the
 * stream.  HB_ERR_NAN for a non-finite Gram matrix. */
int hb_pod_fit(const double* S, const double* B, int64_t ns, int64_t L, int32_t r_max,
               double floor_rel, double* mean, double* basis, double* coef, double* lam,
               int32_t* r_out, void* stream);
/* Host symmetric eigenproblem (no device work): A (host [n][n] row-major,
 * exactly symmetric, read only) = V diag(w) V^T with w (host [n])
 * descending and V (host [n][n] row-major) orthogonal, column k the
 * eigenvector of w[k].  Householder tridiagonalisation, then implicit QR
 * steps with Wilkinson shifts (Golub and Van Loan, ch. 8).  1 <= n <= 4096.
 * HB_ERR_ARG for a non-finite or non-symmetric A; HB_ERR_NOCONV if 30 n QR
 * steps do not converge. */
int hb_sym_eig(int32_t n, const double* A, double* w, double* V);

const char* hb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HB_H */
