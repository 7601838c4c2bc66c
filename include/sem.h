/*
 * sem.h -- C ABI of libsem, an MI355X (gfx950) implementation of the
 * pressure-Poisson solve of the semi-implicit spectral element (SEM)
 * Navier-Stokes method of arXiv 2110.01716 (NekRS on Summit).
 *
 * The discrete problem (Algorithms, eq. field1 and its footnote): on each of
 * E hexahedral elements a field is stored by its values at the (N+1)^3
 * Gauss-Lobatto-Legendre (GLL) points, local index p = i + (N+1) j +
 * (N+1)^2 k with i (the r direction) fastest. The user supplies the nodal
 * coordinates of the isoparametric map of every element and "a global ID for
 * each vertex" (Implementation, Autotuned Communication); nodes with equal IDs
 * are one degree of freedom. Vectors handed to the solver are E-vectors
 * [E][(N+1)^3] in consistent form (every copy of a node holds the same value).
 *
 * Operations:
 *   Ax    local Laplacian A_L u = sum_m D_m^T sum_n G_mn D_n u with six
 *         geometric factors G_mn per point (paper: "Ax", Performance
 *         Measurements, per-kernel profile table);
 *   gs    direct-stiffness summation QQ^T, exchange-and-sum of shared
 *         values (Implementation, Autotuned Communication), with the
 *         homogeneous Dirichlet mask fused in;
 *   pMG   p-multigrid V-cycle with tensor-product interpolation between GLL
 *         levels and Chebyshev-accelerated Jacobi smoothing, run in FP32
 *         (Implementation, pMG paragraph);
 *   solve Jacobi-PCG (Implementation, Helmholtz paragraph) or flexible CG
 *         preconditioned by the pMG V-cycle (Implementation, FlexCG/GMRES
 *         paragraph), outer iteration in FP64.
 *
 * Conventions (all entry points):
 *   - return 0 (SEM_OK) or a negative sem_status; sem_last_error() gives a
 *     thread-local message for the last failure;
 *   - "device" pointers are HIP device allocations on the current device
 *     (e.g. torch tensors on cuda:0); "host" pointers are ordinary memory;
 *   - stream is a hipStream_t (NULL = the default stream). Operations marked
 *     asynchronous only enqueue work; the others return after it finished;
 *   - handles are not thread-safe; distinct handles may be used from distinct
 *     threads on distinct streams;
 *   - a mesh must outlive every pMG hierarchy and batch entry built on it.
 */
#ifndef SEM_H
#define SEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SEM_OK = 0,
  SEM_EINVAL = -1,   /* bad argument, shape or inconsistent mesh data        */
  SEM_EGEOM = -2,    /* Jacobian determinant <= 0 at some GLL point           */
  SEM_ENOMEM = -3,   /* device or host allocation failed, or over the budget  */
  SEM_EHIP = -4,     /* a HIP runtime call failed                             */
  SEM_ENOCONV = -5,  /* iteration limit reached; x holds the last iterate     */
  SEM_ENAN = -6,     /* NaN or Inf met in the right-hand side or an iterate   */
  SEM_EBUSY = -7     /* batch slot table full                                 */
} sem_status;

typedef enum { SEM_F64 = 0, SEM_F32 = 1 } sem_dtype;

typedef struct sem_mesh_s* sem_mesh;
typedef struct sem_pmg_s* sem_pmg;
typedef struct sem_batch_s* sem_batch;

/* ------------------------------------------------------------------------ */
/* Reference element (Algorithms, eq. field1 and footnote)                  */
/* ------------------------------------------------------------------------ */

/* GLL nodes (ascending) and weights of order N, and Dhat_il = h_l'(xi_i)
 * (row-major (N+1)x(N+1)). Host arrays of N+1, N+1 and (N+1)^2 doubles; any
 * may be NULL. SEM_EINVAL if N is outside [1, 15]. */
int sem_reference(int N, double* nodes, double* weights, double* D);

/* Jhat: Lagrange basis on the order-Nc GLL points evaluated at the order-Nf
 * GLL points, row-major (Nf+1)x(Nc+1), host. Used by pMG prolongation
 * (Implementation, pMG paragraph). SEM_EINVAL unless 1 <= Nc, Nf <= 15. */
int sem_interpolation(int Nc, int Nf, double* J);

/* ------------------------------------------------------------------------ */
/* Mesh                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t N;                  /* polynomial order, 1..15                       */
  int64_t E;                  /* number of elements, >= 1                      */
  const double* x;            /* host [E][(N+1)^3] nodal coordinates           */
  const double* y;
  const double* z;
  const int64_t* gid;         /* host [E][(N+1)^3] global node IDs, >= 0        */
  const uint8_t* dirichlet;   /* host [E][(N+1)^3] 1 = homogeneous Dirichlet,
                                 or NULL (pure Neumann)                         */
  void* stream;
} sem_mesh_desc;

typedef struct {
  int32_t N;
  int64_t E;
  int64_t n_local;            /* E (N+1)^3                                    */
  int64_t n_unique;           /* distinct global IDs                          */
  int64_t n_interior;         /* distinct non-Dirichlet IDs                    */
  int64_t n_shared_nodes;     /* distinct IDs with more than one copy          */
  int64_t n_shared_entries;   /* local points belonging to shared IDs          */
  int64_t resident_bytes;     /* device memory owned by the handle             */
  double min_detJ;            /* smallest Jacobian determinant                 */
  double volume;              /* sum of the mass factor B over all points      */
} sem_mesh_info;

/* Copies the host arrays to the device and builds, resident on the device:
 * geometric factors G (6 per point, FP64 and FP32), mass B = W|J|, the
 * gather-scatter map (shared IDs sorted by their first local index, copies in
 * ascending local index), the Dirichlet mask, owner flags for unique-DOF inner
 * products, and the inverse Jacobi diagonal. Synchronous.
 * Errors: SEM_EINVAL (NULL pointer, N or E out of range, gid < 0, more than
 * 2^31-1 local points, Dirichlet flags or coordinates differing between
 * copies of one ID); SEM_EGEOM (det J <= 0; the message names element and
 * point); SEM_ENOMEM; SEM_EHIP. On error *out is NULL. */
int sem_mesh_create(const sem_mesh_desc* desc, sem_mesh* out);
int sem_mesh_destroy(sem_mesh m);
int sem_mesh_query(sem_mesh m, sem_mesh_info* info);

/* Exports resident data to caller-owned device buffers (any may be NULL):
 * G [E][6][(N+1)^3] in the order rr, rs, rt, ss, st, tt; B [E][(N+1)^3];
 * dinv [E][(N+1)^3] = 1/diag(A) on non-Dirichlet copies, 0 on Dirichlet ones
 * (diagonal of the assembled SEM Laplacian). FP64. Asynchronous. */
int sem_mesh_export(sem_mesh m, double* G, double* B, double* dinv, void* stream);

/* Exports the nodal coordinates and global IDs the handle holds (device
 * buffers [E][(N+1)^3], any may be NULL). For the coarse levels of a pMG
 * hierarchy these are the derived coarse coordinates and IDs. Asynchronous. */
int sem_mesh_export_nodes(sem_mesh m, double* x, double* y, double* z, int64_t* gid,
                          uint8_t* dirichlet, void* stream);

/* Local Poisson operator on elements [e0, e0+ne): Au = A_L u, no gather-scatter
 * and no mask (the paper's element-local "Ax" kernel). u, Au: device [E][Np]
 * of dtype t; elements outside the range are not touched. FP32 uses the
 * FP32-rounded G. Asynchronous. SEM_EINVAL on a bad range or dtype. */
int sem_ax(sem_mesh m, sem_dtype t, const void* u, void* Au, int64_t e0, int64_t ne, void* stream);

/* Helmholtz variant (A_L + lambda B) u on all elements (velocity substep
 * operator, Implementation, Helmholtz paragraph). Asynchronous. */
int sem_helmholtz(sem_mesh m, sem_dtype t, const void* u, void* Au, double lambda, void* stream);

/* In place v <- M QQ^T v (apply_mask != 0) or v <- QQ^T v: every copy of a
 * shared ID receives the sum of all copies, summed in ascending local-index
 * order. Device [E][Np] of dtype t. Asynchronous. */
int sem_gs(sem_mesh m, sem_dtype t, void* v, int apply_mask, void* stream);

/* Local mass: Bu = B u pointwise. Asynchronous. */
int sem_mass(sem_mesh m, sem_dtype t, const void* u, void* Bu, void* stream);

/* Unique-DOF inner product sum over distinct IDs of a*b of two consistent
 * E-vectors; result written to *result (host). Deterministic (fixed reduction
 * order). Synchronous. */
int sem_dot(sem_mesh m, sem_dtype t, const void* a, const void* b, double* result, void* stream);

/* sem_dot for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same product with its partial sums kept in a static device array of the
 * library (1 MiB per device, held until the process ends) instead of a
 * buffer allocated per call; the sum of the partials is reduced on the device
 * in a fixed order, so the result can differ from sem_dot's in the last bits.
 * Makes no device allocation. The current device must be the mesh's. Limit:
 * n_local <= 134,217,728 (2^27) local points, else SEM_EINVAL. Calls that
 * overlap on one device share the array and race. Synchronous. */
int sem_dot_noalloc(sem_mesh m, sem_dtype t, const void* a, const void* b, double* result, void* stream);

/* ------------------------------------------------------------------------ */
/* p-multigrid (Implementation, pMG paragraph)                               */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t n_levels;           /* 2..8; 0 = default {N, (N-1)/2, 1} (or {N,1}) */
  int32_t orders[8];          /* strictly decreasing, orders[0] = N, last = 1  */
  sem_dtype smoother_dtype;   /* SEM_F32 (default) or SEM_F64                  */
  int32_t cheb_degree;        /* Chebyshev degree per sweep (default 2)        */
  int32_t pre, post;          /* sweeps per level (default 1, 1)               */
  double eig_lo, eig_hi;      /* interval [lo rho, hi rho] (0.1, 1.1)          */
  int32_t power_iters;        /* power iterations for rho (20)                 */
  const double* rho_override; /* host, one per smoothed level, or NULL         */
  double coarse_rtol;         /* coarse Jacobi-PCG tolerance (1e-2)            */
  int32_t coarse_maxit;       /* coarse iteration cap (500)                    */
  int32_t coarse_fixed_iters; /* > 0: exactly this many coarse iterations      */
  int32_t coarse_check_every; /* coarse convergence polled every k iters (8)   */
  int32_t smoother;           /* SEM_SMOOTH_* (default Chebyshev-Jacobi)       */
} sem_pmg_opts;

/* pMG smoothers (Implementation, pMG paragraph): Chebyshev acceleration of
 * point Jacobi, or of overlapping Schwarz with fast-diagonalization local
 * solves on elements extended by one node layer across each face (eq. fdm),
 * additive (ASM, counting weights) or restricted (RAS, own nodes only). */
enum {
  SEM_SMOOTH_CHEB_JACOBI = 0,
  SEM_SMOOTH_CHEB_ASM = 1,
  SEM_SMOOTH_CHEB_RAS = 2
};

/* Fills o with the defaults above (n_levels = 0 meaning the default schedule). */
void sem_pmg_opts_default(sem_pmg_opts* o);

/* Test hook: z = M r with the preconditioner the smoother accelerates at a
 * smoothed level: D^-1 (Chebyshev-Jacobi) or W S, S = sum_e R_e^T A~_e^-1 R_e
 * by fast diagonalization (eq. fdm) and W the ASM counting or RAS averaging
 * weights (masked). r, z: device [E][Np] of that level in the smoother dtype,
 * r consistent and masked. Synchronous. SEM_EINVAL on the coarsest level. */
int sem_pmg_smoother_apply(sem_pmg p, int level, const void* r, void* z, void* stream);

typedef struct {
  int32_t n_levels;
  int32_t orders[8];
  double rho[8];              /* largest eigenvalue estimate of D^-1 A per level */
  int64_t n_unique[8];
  int64_t resident_bytes;
} sem_pmg_info;

/* Builds the level hierarchy on the device: coarse nodal coordinates by
 * evaluating each element's isoparametric map at the coarse GLL points,
 * coarse global IDs from mesh entities (vertex, edge, face, interior) keyed by
 * the fine IDs, coarse masks, geometric factors, Jacobi diagonals and rho by
 * power iteration from a splitmix64 start vector keyed by global ID.
 * Synchronous. SEM_EINVAL on a bad schedule. */
int sem_pmg_setup(sem_mesh m, const sem_pmg_opts* o, sem_pmg* out);
int sem_pmg_destroy(sem_pmg p);
int sem_pmg_query(sem_pmg p, sem_pmg_info* info);

/* Level l (0 = finest) as a mesh handle owned by the hierarchy (do not
 * destroy). Lets sem_ax/sem_gs/sem_mesh_export act on coarse levels. */
int sem_pmg_level(sem_pmg p, int level, sem_mesh* out);

/* Transfers between level l and l+1 (device E-vectors of the smoother dtype
 * for levels that are smoothed, FP64 for the coarsest):
 *   direction 0 (prolong):  out_fine += (J x J x J) in_coarse, element-wise;
 *   direction 1 (restrict): out_coarse = M QQ^T (J^T x J^T x J^T)(w . in_fine)
 *     with w the owner flag of each fine copy (transpose of prolongation in
 *     the unique-DOF inner product). Asynchronous. */
int sem_pmg_transfer(sem_pmg p, int level, int direction, const void* in, void* out, void* stream);

/* One V-cycle z = M_pMG(r) on consistent masked FP64 E-vectors of the finest
 * level (device). Synchronous. */
int sem_pmg_apply(sem_pmg p, const double* r, double* z, void* stream);

/* ------------------------------------------------------------------------ */
/* Solvers                                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
  double rtol;                /* stop when ||r|| <= rtol ||b|| (1e-8)          */
  int32_t maxit;              /* outer iteration cap (10000)                    */
  int32_t check_every;        /* host polls convergence every k iters (1)       */
  int32_t fixed_iters;        /* > 0: exactly this many iterations, no test     */
  double lambda;              /* Helmholtz shift: solve (A + lambda B) x = b, the
                                 velocity-substep operator (Implementation,
                                 Helmholtz paragraph); Jacobi-PCG only (the
                                 hierarchy must be NULL); 0 = Poisson          */
} sem_solve_opts;

void sem_solve_opts_default(sem_solve_opts* o);

typedef struct {
  int32_t iters;              /* outer iterations performed                     */
  int32_t status;             /* sem_status of this solve                       */
  double relres;              /* recurrence residual ||r|| / ||b||              */
  double relres_true;         /* ||b - A x|| / ||b|| recomputed at exit         */
  int64_t coarse_iters;       /* total coarse-grid PCG iterations               */
  double seconds;             /* wall time of the solve call                    */
  double relres_initial;      /* ||b - A x0|| / ||b|| of the starting guess: 1
                                 for x0 = 0, smaller after projection           */
  int64_t launches;           /* kernels queued for the solve from its start to
                                 its completion, one per phase of an iteration;
                                 in a batched or continuous-batching call the
                                 launches are shared by the problems in flight,
                                 so the last problem to finish reports the
                                 whole call. Projected solves report their
                                 inner solve's; GMRES reports 0 (not counted) */
} sem_solve_info;

/* Solves A x = b, A the assembled masked SEM Laplacian, with Jacobi-PCG
 * (p == NULL) or flexible CG preconditioned by one pMG V-cycle per iteration
 * (p != NULL). b, x: device FP64 [E][Np], consistent and masked; x is
 * overwritten (x0 = 0). Residual norms are unique-DOF 2-norms. Returns when
 * converged (SEM_OK), at maxit (SEM_ENOCONV, x = last iterate) or on NaN
 * (SEM_ENAN). b = 0 returns x = 0 after 0 iterations. info may be NULL. */
int sem_pcg_solve(sem_mesh m, sem_pmg p, const double* b, double* x, const sem_solve_opts* o,
                  sem_solve_info* info, void* stream);

/* n independent solves advanced together: each phase of an iteration is one
 * launch over all unfinished problems. p[i] may be NULL (Jacobi-PCG) but all
 * problems must then use the same solver kind. Results are identical to n
 * separate sem_pcg_solve calls (per-problem reductions in a fixed order). */
int sem_pcg_solve_batched(int n, const sem_mesh* m, const sem_pmg* p, const double* const* b,
                          double* const* x, const sem_solve_opts* o, sem_solve_info* info,
                          void* stream);

/* Device bytes a solve on (m, p) allocates for its vectors. */
size_t sem_solve_workspace_bytes(sem_mesh m, sem_pmg p);

/* Solves A x = b (or (A + lambda B) x = b with the Jacobi preconditioner)
 * by right-preconditioned flexible GMRES(K) (Implementation, FlexCG/GMRES
 * paragraph; Performance Results, GMRES with K <= 6): preconditioner one pMG
 * V-cycle (p != NULL) or Jacobi (p == NULL). Each Arnoldi step takes one
 * round of classical Gram-Schmidt with a single multi-dot; the least-squares
 * residual (Givens rotations) is the convergence test; after K steps without
 * convergence it restarts from the true residual. K in [1, 64]; o->maxit
 * bounds the total number of steps, o->fixed_iters runs exactly that many.
 * b, x: device FP64 [E][Np], consistent and masked; x0 = 0. Device memory:
 * 2K + 2 FP64 E-vectors from the workspace pool. Errors as sem_pcg_solve. */
int sem_gmres_solve(sem_mesh m, sem_pmg p, int K, const double* b, double* x, const sem_solve_opts* o,
                    sem_solve_info* info, void* stream);

/* ------------------------------------------------------------------------ */
/* Projection onto prior solutions (Implementation, "Projection Is Key")     */
/* ------------------------------------------------------------------------ */

/* A space of up to L_max earlier solutions kept A-orthonormal on the device
 * (P and AP, 2 (L_max + 1) FP64 E-vectors). For a new b the best approximation in
 * the A-norm is xbar = P P^T b (one multi-dot); the Krylov solver then solves
 * A dx = b - A xbar; dx is A-orthogonalised against P by one round of
 * classical Gram-Schmidt (one multi-dot) and appended. When the space is full
 * it restarts from the latest solution alone. */
typedef struct sem_proj_s* sem_proj;
int sem_proj_create(sem_mesh m, int L_max, sem_proj* out);
int sem_proj_destroy(sem_proj pr);
/* Number of vectors currently in the space. */
int sem_proj_size(sem_proj pr, int* L);
/* Empties the space. */
int sem_proj_reset(sem_proj pr);
/* Inner solver of sem_pcg_solve_projected: K = 0 (default) the CG family of
 * sem_pcg_solve, K > 0 flexible GMRES(K) as sem_gmres_solve. */
int sem_proj_set_gmres(sem_proj pr, int K);
/* Exports basis vector i (device FP64 [E][Np] buffers p and Ap, either may be
 * NULL). SEM_EINVAL if i >= size. Asynchronous. */
int sem_proj_export(sem_proj pr, int i, double* p, double* Ap, void* stream);

/* sem_pcg_solve with the projected starting guess; the residual test stays
 * relative to ||b||; info->relres_initial reports the projected residual.
 * The solution is then added to the space. The mesh must be the one the
 * space was created on. */
int sem_pcg_solve_projected(sem_proj pr, sem_pmg p, const double* b, double* x, const sem_solve_opts* o,
                            sem_solve_info* info, void* stream);

/* ------------------------------------------------------------------------ */
/* Continuous batching: solves join and leave at iteration boundaries        */
/* ------------------------------------------------------------------------ */

/* A batch holds up to max_slots active solves (pMG-preconditioned flexible CG
 * if the slot has a hierarchy, else Jacobi-PCG), all advanced together by
 * sem_batch_step. Each solve's arithmetic depends only on its own data, so a
 * result is the same alone or in any mix. */
int sem_batch_create(int max_slots, void* stream, sem_batch* out);
int sem_batch_destroy(sem_batch b);

/* Admits a solve into a free slot (allocates its workspace, computes ||b||,
 * sets x = 0). Returns the slot index in *slot. SEM_EBUSY if no slot is free,
 * SEM_ENOMEM if the workspace does not fit. b and x must stay valid until the
 * slot is released. */
int sem_batch_add(sem_batch b, sem_mesh m, sem_pmg p, const double* rhs, double* x,
                  const sem_solve_opts* o, int* slot);

/* Runs `iters` iterations of every active, unfinished solve and polls their
 * convergence. *n_active receives the number still running. */
int sem_batch_step(sem_batch b, int iters, int* n_active);

/* Status of a slot: info->status is 1 while running, else the final status. */
int sem_batch_poll(sem_batch b, int slot, sem_solve_info* info);

/* Frees the slot's workspace (finished or not). */
int sem_batch_release(sem_batch b, int slot);

/* ------------------------------------------------------------------------ */

/* ------------------------------------------------------------------------ */
/* Bandwidth probe (Performance Measurements: each kernel is rated against   */
/* the realizable memory bandwidth that a STREAM triad reaches, and counts   */
/* as roofline performance above 70% of it)                                 */
/* ------------------------------------------------------------------------ */

/* dst[i] = src[0][i] + s * sum_{k=1}^{n_in-1} src[k][i] for 0 <= i < n.
 * src: device, n_in contiguous arrays of n doubles ([n_in][n]); dst: device,
 * n doubles; both caller-owned, 16-byte aligned, not overlapping. n_in = 1 is
 * a copy, n_in = 2 the STREAM triad a = b + s c, n_in = 7 the FP64 local
 * Laplacian's read:write mix (seven streams in, one out). 1 <= n_in <= 8, n
 * even and >= 0 (n = 0 does nothing); otherwise SEM_EINVAL. Asynchronous. */
int sem_stream(int n_in, const double* src, double* dst, double s, int64_t n, void* stream);

const char* sem_status_string(int status);
const char* sem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SEM_H */
