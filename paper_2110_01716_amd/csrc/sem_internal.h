// Internal declarations shared by the libsem sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <new>
#include <cstdio>
#include <string>
#include <vector>

#include "sem.h"

namespace sem {

constexpr int kMaxN = 15;
constexpr int kMaxNP = kMaxN + 1;
constexpr int kMaxLevels = 8;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Error {
  int code;
};
void set_error(const char* fmt, ...);
[[noreturn]] void fail(int code, const char* fmt, ...);

#define SEM_HIP(call)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      ::sem::fail(e_ == hipErrorOutOfMemory ? SEM_ENOMEM : SEM_EHIP, "%s: %s (%s:%d)",   \
                  #call, hipGetErrorString(e_), __FILE__, __LINE__);                      \
  } while (0)

// C-ABI wrapper: runs f, turns sem::Error into its status code.
template <typename F>
int guarded(F&& f) {
  try {
    f();
    return SEM_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host memory exhausted");
    return SEM_ENOMEM;
  } catch (const std::exception& e) {
    set_error("internal error: %s", e.what());
    return SEM_EHIP;
  } catch (...) {  // nothing crosses the C ABI
    set_error("internal error: unknown exception");
    return SEM_EHIP;
  }
}

// ---------------------------------------------------------------------------
// reference element (host, FP64)
// ---------------------------------------------------------------------------
void gll_points(int N, double* x, double* w);
void deriv_matrix(int N, double* D);  // row-major (N+1)x(N+1)
void lagrange_matrix(int n_src, const double* src, int n_dst, const double* dst, double* M);

// 1D matrix passed by value to kernels (copied to LDS there).
template <typename T>
struct Mat1D {
  T a[kMaxNP * kMaxNP];
};

// ---------------------------------------------------------------------------
// device memory helper
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t n);
  void release();
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------------------
// one mesh level, resident on the device
// ---------------------------------------------------------------------------
struct MeshData {
  int N = 0, NP = 0, Np = 0;
  int64_t E = 0, nloc = 0;
  int64_t n_unique = 0, n_interior = 0, n_shared = 0, n_shared_entries = 0, n_dir_single = 0;
  double min_detJ = 0, volume = 0;
  std::vector<double> D;   // (N+1)^2 host copy
  std::vector<double> w;   // GLL weights
  DevBuf Dg64, Dg32, wg;   // device copies of Dhat (FP64, FP32) and the weights
  DevBuf x, y, z;          // double [nloc]
  DevBuf gid;              // int64 [nloc]
  DevBuf dmask;            // uint8 [nloc]  1 = Dirichlet copy
  DevBuf owner;            // uint8 [nloc]  1 = first copy of its ID (0 on Dirichlet)
  DevBuf G64, G32;         // [E][6][Np]
  DevBuf B64, B32;         // [E][Np]
  DevBuf dinv64, dinv32;   // [nloc]
  DevBuf gs_off;           // int32 [n_shared+1]
  DevBuf gs_idx;           // int32 [n_shared_entries]
  DevBuf gs_dir;           // uint8 [n_shared]  1 = Dirichlet node
  DevBuf dir_idx;          // int32 [n_dir_single]  Dirichlet copies of unshared IDs
  // assembled form on unique DOFs (coarsest pMG level only)
  bool assembled = false;
  int ell_w = 0;           // ELL width (longest row)
  DevBuf umap;             // int32 [nloc]  unique index of each copy
  DevBuf u2l_off;          // int32 [n_unique+1]  copies of each unique DOF (CSR)
  DevBuf u2l_idx;          // int32 [nloc]  local indices, ascending within a DOF
  DevBuf udir;             // uint8 [n_unique]  Dirichlet DOF
  DevBuf dinv_u;           // f64 [n_unique]  inverse diagonal, 0 on Dirichlet
  DevBuf ell_col;          // int32 [W][n_unique]
  DevBuf ell_val;          // f64 [W][n_unique]
  int64_t resident_bytes() const;
};

}  // namespace sem

struct sem_mesh_s {
  sem::MeshData d;
  bool owned_by_pmg = false;
};

namespace sem {

// ---------------------------------------------------------------------------
// kernel argument tables: a launch covers one problem (inline args) or many
// (device array of args + block prefix `starts[n+1]`)
// ---------------------------------------------------------------------------
template <typename A>
struct Table {
  A one;
  const A* many = nullptr;
  const int* starts = nullptr;
  int n = 0;
};

// skip flags: a problem's launch does nothing when either flag is nonzero
struct Skip {
  const int* f0 = nullptr;
  const int* f1 = nullptr;
};

template <typename T>
struct AxArgs {
  const T* G = nullptr;
  const T* B = nullptr;   // Helmholtz mass factor, or null
  const T* u = nullptr;
  T* Au = nullptr;
  int64_t e0 = 0, ne = 0;
  double lambda = 0;
  double* partial = nullptr;  // per block: sum u . Au over the block's points
  Skip skip;
};

template <typename T>
struct GsArgs {
  T* v = nullptr;
  const int* off = nullptr;
  const int* idx = nullptr;
  const uint8_t* sdir = nullptr;
  const int* dir_idx = nullptr;
  int64_t n_shared = 0, n_dir = 0;
  int mask = 1;
  Skip skip;
};

enum VecOp : int {
  V_PCG_UPDATE = 0,   // x += a p; r -= a w; partial0 = own r.r; partial1 = own r.dinv.r (Jacobi)
  V_P_JACOBI,         // p = dinv r + beta p
  V_P_FLEX,           // p = z + beta p
  V_DOT2,             // partial0 = own z.w ; partial1 = own r.z
  V_DOT1,             // partial0 = own r.r  (r = x slot a)
  V_RZ_JACOBI,        // partial0 = own r.dinv.r ; p = dinv r
  V_CHEB_INIT0,       // d = dinv r / theta; x = d           (pre-smoothing start)
  V_CHEB_INITX,       // res = r - t; d = dinv res / theta; x += d
  V_CHEB_STEP,        // res -= t; d = c1 d + c2 dinv res; x += d
  V_CHEB_STEP0,       // first step after INIT0: res = r - t; d = c1 d + c2 dinv res; x += d
  // fused Chebyshev-Jacobi variants (no writes that nothing reads):
  V_CHEB_INIT0D,      // d = c0 dinv r                         (x = d left implicit)
  V_CHEB_INIT0D_IN64, // r = (T) in64; d = c0 dinv r            (V-cycle entry cast folded in)
  V_CHEB_STEP0X,      // after INIT0D: res = r - t; dn = c1 d + c2 dinv res; x = d + dn; d = dn
  V_CHEB_LAST0X,      // after INIT0D, last step: x = d + c1 d + c2 dinv (r - t)
  V_CHEB_LAST,        // last step: x += c1 d + c2 dinv (res - t)
  V_CHEB_LAST_OUT64,  // last step, V-cycle exit: out64 = (double)(x + c1 d + c2 dinv (res - t));
                      //   partial0 = own out64 . w64, partial1 = own out64 . r64
  V_CHEB_INITX_LAST,  // degree 1 from x: x += c0 dinv (r - t)
  V_CHEB_INITX_OUT64, // degree 1 from x, V-cycle exit: out64 = (double)(x + c0 dinv (r - t)); partials as above
  V_RES0,             // res = r - t
  V_RES,              // res -= t
  V_CHEB_UPD,         // d = c1 d + c2 dinv r; x += d   (r: a smoother's preconditioned residual)
  V_CHEB_UPD0,        // d = c2 dinv r; x += d
  V_CHEB_UPD_OUT64,   // last Schwarz step, V-cycle exit: out64 = (double)(x + c1 d + c2 dinv r); partials as above
  V_CHEB_UPD0_OUT64,  // degree 1: out64 = (double)(x + c2 dinv r); partials as above
  V_ZERO,             // x = 0
  V_FILL,             // x = c0
  V_COPY,             // x = r
  V_SCALE_DINV,       // x = dinv * r
  V_NORMALIZE,        // x = r * scal[S_TMP]
  V_TRUE_RES,         // partial0 = own (r - t).(r - t)
  V_DIV_DINV,         // x = r / dinv (0 where dinv = 0)
  V_SCALE,            // x = c0 r
  V_AXPY,             // x += c0 r
  V_COUNT
};

// scalar slots of a solve stage (per problem, device doubles)
enum Scal : int {
  S_BB = 0, S_RZ, S_PW, S_ALPHA, S_BETA, S_RR, S_RELRES, S_ZW, S_TMP, S_RZ_NEW, S_COUNT
};
// integer flags of a solve stage
// F_ITERS2: second slot of the coarse iteration counter (two-launch coarse CG)
enum Flag : int { F_DONE = 0, F_STATUS, F_ITERS, F_TOTAL, F_ITERS2, F_COUNT };

template <typename T>
struct VecArgs {
  int64_t n = 0;
  T* x = nullptr;
  T* r = nullptr;
  T* p = nullptr;
  T* w = nullptr;
  T* z = nullptr;
  T* t = nullptr;
  T* res = nullptr;
  T* d = nullptr;
  const T* dinv = nullptr;
  const uint8_t* owner = nullptr;
  const double* scal = nullptr;
  double* partial = nullptr;  // [2][stride]
  int64_t stride = 0;
  double c0 = 0, c1 = 0, c2 = 0;
  const double* in64 = nullptr;  // V_CHEB_INIT0D_IN64; the *_OUT64 ops read it as r64
  double* out64 = nullptr;       // V_CHEB_*_OUT64
  const double* w64 = nullptr;   // V_CHEB_*_OUT64: partials of out64 . w64 and out64 . r64 (the FlexCG dots)
  Skip skip;
};

template <typename Tin, typename Tout>
struct CastArgs {
  int64_t n = 0;
  const Tin* in = nullptr;
  Tout* out = nullptr;
  Skip skip;
};

enum FinOp : int {
  FIN_INIT = 0,       // bb = s0; rr = bb; detect zero / NaN rhs
  FIN_RZ,             // rz = s0; beta = 0
  FIN_ALPHA,          // pw = s0; alpha = rz / pw
  FIN_CHECK,          // rr = s0; iters++; convergence test
  FIN_CHECK_JACOBI,   // as FIN_CHECK plus beta = s1 / rz, rz = s1
  FIN_BETA_FLEX,      // zw = s0, rz_new = s1; beta = -alpha zw / rz; rz = rz_new
  FIN_NORM,           // tmp = 1 / sqrt(s0)
  FIN_STORE           // tmp = s0
};

struct FinArgs {
  const double* partial = nullptr;  // [2][stride]
  int64_t stride = 0;
  int64_t nblk = 0;
  double* scal = nullptr;
  int* flags = nullptr;
  double rtol = 0;
  int maxit = 0;
  int fixed = 0;
  int* total = nullptr;             // optional counter incremented with iters (coarse total)
  Skip skip;
};

template <typename Tf, typename Tc>
struct XferArgs {
  int64_t E = 0;
  const int* umap_c = nullptr;  // prolong from a unique-DOF coarse vector: zc[umap_c[local]]
  // restrict: out_c = (J^T)^3 ((rf - tf) . owner_f)   (tf may be null)
  const Tf* rf = nullptr;
  const Tf* tf = nullptr;
  const uint8_t* owner_f = nullptr;
  Tc* out_c = nullptr;
  // prolong: xf += J^3 zc
  const Tc* zc = nullptr;
  Tf* xf = nullptr;
  Skip skip;
};

// out[r] = 0 on Dirichlet DOFs, else sum of the local copies of DOF r (Q^T)
struct UsumArgs {
  int64_t n = 0;
  const int* off = nullptr;
  const int* idx = nullptr;
  const uint8_t* udir = nullptr;
  const double* in = nullptr;
  double* out = nullptr;
  Skip skip;
};

// Overlapping Schwarz smoother, one block per element (N+3)^3 extended box.
// desc [E][6][8] int32 per face: {nbr, g_off, g_su, g_sv, p_off, p_su, p_sv, kind}:
//   the extension value for face node (u, v) is in[nbr*Np + g_off + u*g_su + v*g_sv];
//   the element's depth-1 node (u, v) behind the face receives
//   ovl[nbr*6*NP^2 + p_off + u*p_su + v*p_sv]; kind 0 neighbour, 1 Dirichlet, 2 Neumann.
// S [E][3][NE][NE] (row: ext index, column: mode), lam [E][3][NE].
// mode 0: fast-diagonalization solve; mode 1: identity on the active positions
// (the counting function). out: own (N+1)^3 block; ovl [E][6][NP^2] (face
// layers of the local solution, v*NP + u), skipped when null (RAS).
template <typename T>
struct SchwarzArgs {
  int64_t E = 0;
  const T* in = nullptr;
  T* out = nullptr;
  T* ovl = nullptr;
  const int* desc = nullptr;
  const T* S = nullptr;
  const T* lam = nullptr;
  Skip skip;
};
// out[e][depth-1 node behind face f] += pulled overlap of the neighbour across f
template <typename T>
struct SchwarzPullArgs {
  int64_t E = 0;
  T* out = nullptr;
  const T* ovl = nullptr;
  const int* desc = nullptr;
  Skip skip;
};
// per element: 8 corner global IDs (lexicographic i, j, k), 6 face flags
// (1 = every node of the face is Dirichlet), 3 mean lengths (r, s, t)
struct SchwarzInfoArgs {
  int N = 0;
  int64_t E = 0;
  const double *x = nullptr, *y = nullptr, *z = nullptr;
  const int64_t* gid = nullptr;
  const uint8_t* dmask = nullptr;
  int64_t* corners = nullptr;
  uint8_t* face_dir = nullptr;
  double* lengths = nullptr;
};

// Coarse-grid Jacobi-PCG on the unique DOFs of an assembled level in two
// launches per iteration and no finalize launch (parity `par` alternates the
// ring slots of rz and of the iteration counter, so no launch overwrites a
// value its own blocks read):
//  k_cg_pspmv:  every block reduces the previous update's partials (r.r,
//               r.z) in a fixed order, tests convergence, forms beta; then
//               q = A z, p = z + beta p, w = q + beta w row by row, partial p . w
//  k_cg_update: every block reduces the p . w partials, alpha = rz / pw;
//               x += alpha p, r -= alpha w, z = D^-1 r, partials r.r and r.z
struct CgArgs {
  int64_t n = 0;
  int W = 0;
  const int* col = nullptr;
  const double* val = nullptr;
  const double* dinv = nullptr;
  double* x = nullptr;
  double* r = nullptr;
  double* w = nullptr;
  double* p = nullptr;
  double* z = nullptr;        // D^-1 r (written by the update, gathered by the SpMV)
  double* partial = nullptr;  // regions 0: r.r, 1: r.D^-1 r (update), 2: p.w (spmv)
  int64_t stride = 0;
  int64_t nblk_upd = 0;       // blocks of k_cg_update (partials in regions 0, 1)
  int64_t nblk_sp = 0;        // blocks of k_cg_pspmv (partials in region 2)
  double* scal = nullptr;     // coarse stage scalars (S_BB, ring S_RZ / S_RZ_NEW, ...)
  int* flags = nullptr;       // coarse stage flags (ring F_ITERS / F_ITERS2, ...)
  int* total = nullptr;       // outer stage F_TOTAL (coarse iterations of the solve)
  int par = 0;
  double rtol = 0;
  int maxit = 0;
  int fixed = 0;
  Skip skip;
};

// multi-dot: partial[k][blk] = sum over owned points of v[k] . y (k < K)
struct MdotArgs {
  int64_t n = 0;
  int K = 0;
  const double* const* v = nullptr;  // device array of K vector pointers
  const double* y = nullptr;
  const uint8_t* owner = nullptr;
  double* partial = nullptr;         // [K][stride]
  int64_t stride = 0;
};
// out = scale * (a0 y + sign sum_k coef[k] v[k]), coef on the device
struct LincombArgs {
  int64_t n = 0;
  int K = 0;
  const double* const* v = nullptr;
  const double* coef = nullptr;
  const double* y = nullptr;
  double a0 = 0, sign = 1, scale = 1;
  double* out = nullptr;
};

// ---------------------------------------------------------------------------
// launchers (defined in sem_kernels.hip)
// ---------------------------------------------------------------------------
int ax_blocks(int N, int64_t ne, bool f32 = false);  // f32: blocks of the FP32 kernel
int64_t vec_blocks(int64_t n);
int64_t gs_blocks(int64_t n_shared, int64_t n_dir);
int xfer_blocks(int Nf, int Nc, int64_t E);
constexpr int kFinThreads = 1024;

// helm: the table's problems carry B and lambda (Helmholtz (A_L + lambda B) u)
template <typename T>
void launch_ax(int N, const Table<AxArgs<T>>& t, int64_t total_blocks, const T* D, hipStream_t s,
               bool helm = false);
template <typename T>
void launch_gs(const Table<GsArgs<T>>& t, int64_t total_blocks, hipStream_t s);
template <typename T>
void launch_vec(VecOp op, const Table<VecArgs<T>>& t, int64_t total_blocks, hipStream_t s);
template <typename Tin, typename Tout>
void launch_cast(const Table<CastArgs<Tin, Tout>>& t, int64_t total_blocks, hipStream_t s);
void launch_fin(FinOp op, const Table<FinArgs>& t, int nprob, hipStream_t s);
int64_t spmv_blocks(int64_t n);
void launch_mdot(const MdotArgs& a, hipStream_t s);            // grid: vec_blocks(n) x ceil(K/8)
void launch_mfin(const double* partial, int64_t stride, int64_t nblk, int K, double* out, hipStream_t s);
void launch_lincomb(const LincombArgs& a, hipStream_t s);
int schwarz_blocks(int64_t E);  // one block per element
template <typename T>
void launch_schwarz(int N, int mode, const Table<SchwarzArgs<T>>& t, int64_t total_blocks, hipStream_t s);
template <typename T>
void launch_schwarz_pull(int N, const Table<SchwarzPullArgs<T>>& t, int64_t total_blocks, hipStream_t s);
void launch_schwarz_info(const SchwarzInfoArgs& a, hipStream_t s);
int64_t cg_update_blocks(int64_t n);
void launch_cg_update(const Table<CgArgs>& t, int64_t total_blocks, hipStream_t s); // blocks: cg_update_blocks(n)
// p update and w = A p in one launch (p_old != p_new); blocks: cg_update_blocks(n)
void launch_cg_pspmv(const Table<CgArgs>& t, int64_t total_blocks, hipStream_t s);
void launch_usum(const Table<UsumArgs>& t, int64_t total_blocks, hipStream_t s);
template <typename Tf, typename Tc>
void launch_xfer(int dir, int Nf, int Nc, const Table<XferArgs<Tf, Tc>>& t, int64_t total_blocks,
                 const double* J, hipStream_t s);

// setup kernels
void launch_geometry(const MeshData& m, double* detmin_partial, double* vol_partial, int64_t* bad_index,
                     hipStream_t s);
void launch_diag_local(const MeshData& m, double* dl, hipStream_t s);
void launch_dinv_finish(const MeshData& m, const double* d_assembled, hipStream_t s);
// out = 0 on Dirichlet copies, else 1 / d
void launch_dinv_to(const MeshData& m, const double* d_assembled, double* out, hipStream_t s);
void launch_tensor_coords(int Nf, int Nc, int64_t E, const double* in, double* out, const double* Jcf,
                          hipStream_t s);
void launch_start_vector(int64_t n, const int64_t* gid, const uint8_t* dmask, double* v, hipStream_t s);
void launch_mass(int N, int64_t nloc, int is_f32, const void* B, const void* u, void* Bu, hipStream_t s);

// gather-scatter map construction (sem_gsmap.hip)
void build_gs_map(MeshData& m, hipStream_t s);
// assembled unique-DOF operator (sem_assemble.hip)
void build_assembled(MeshData& m, hipStream_t s);

// mesh construction from device coordinates and host IDs/flags (sem_mesh.cpp)
void build_mesh(MeshData& m, int N, int64_t E, const int64_t* gid_host, const uint8_t* dir_host,
                hipStream_t s);

// deterministic dot product on one mesh (FP64 result), synchronous
double mesh_dot(const MeshData& m, sem_dtype t, const void* a, const void* b, hipStream_t s);

// single-problem helpers used by setup code
void apply_A(const MeshData& m, sem_dtype t, const void* u, void* Au, hipStream_t s);
// (M QQ^T (A_L + lambda B)) u in FP64
void apply_H(const MeshData& m, double lambda, const double* u, double* Hu, hipStream_t s);
// inverse Jacobi diagonal of M QQ^T (A_L + lambda B) into out (FP64), using tmp [nloc]
void helmholtz_dinv(const MeshData& m, double lambda, double* out, double* tmp, hipStream_t s);
// QQ^T (and the Dirichlet mask if mask != 0) in place, FP64 or FP32
void mesh_gs(const MeshData& m, sem_dtype t, void* v, int mask, hipStream_t s);
// FP64 unique-DOF inner product with caller scratch partial [2 * vec_blocks(nloc)]
double mesh_dot_ws(const MeshData& m, const double* a, const double* b, double* partial, hipStream_t s);
// out[k] = (v_k, y) over unique DOFs for k < K; v is a device array of K
// vector pointers; partial [K][stride] scratch, stride >= vec_blocks(nloc)
void mesh_multidot(const MeshData& m, const double* const* v, int K, const double* y, double* partial,
                   int64_t stride, double* out, hipStream_t s);
// out = scale (a0 y + sign sum_{k<K} coef[k] v_k), coef on the device; out may alias y or v_k
void mesh_lincomb(const MeshData& m, const double* const* v, int K, const double* coef, const double* y, double a0,
                  double sign, double scale, double* out, hipStream_t s);
// single-vector FP64 update x <- op(x, r, c0) over n entries (V_SCALE, V_AXPY, V_SCALE_DINV, ...)
void vec_op1(VecOp op, int64_t n, double* x, const double* r, double c0, const double* dinv, hipStream_t s);

// workspace pool shared by all solves (reuses freed device blocks)
void* pool_get(size_t bytes);
void pool_put(void* p, size_t bytes);

// One pMG V-cycle z = M(r) on FP64 consistent E-vectors, with the solver
// engine's plan built once and reused across applications.
struct VcycleRunner;
VcycleRunner* vcycle_runner_create(sem_pmg p, hipStream_t s);
void vcycle_runner_apply(VcycleRunner* v, const double* r, double* z);
int64_t vcycle_runner_coarse_iters(VcycleRunner* v);
void vcycle_runner_destroy(VcycleRunner* v);

}  // namespace sem

// ---------------------------------------------------------------------------
// p-multigrid hierarchy
// ---------------------------------------------------------------------------
namespace sem {
// overlapping Schwarz data of one smoothed level (layouts as in SchwarzArgs)
struct SchwarzData {
  bool on = false;
  bool ras = false;
  DevBuf desc;                   // int32 [E][6][8]
  DevBuf S64, L64, S32, L32;     // FDM eigenvectors / eigenvalues
  DevBuf w64, w32;               // weights: 1 / counting function (ASM) or 1 / multiplicity (RAS)
};

struct PmgLevel {
  sem_mesh_s* mesh = nullptr;    // level mesh (level 0: the user's mesh)
  double rho = 0, theta = 0, delta = 0;
  std::vector<double> c1, c2;    // Chebyshev step coefficients, steps 1..k-1
  DevBuf J;                      // prolongation from level l+1: (N_l+1) x (N_{l+1}+1)
  DevBuf JT;                     // restriction to level l+1:   (N_{l+1}+1) x (N_l+1)
  SchwarzData sw;
};
// builds the Schwarz data of a level (sem_schwarz.cpp)
void schwarz_setup(const MeshData& m, bool ras, SchwarzData& sw, hipStream_t s);
// z = W S(r) in FP64 or FP32 (the smoother's preconditioner); tmp_ovl [E][6][NP^2] of the same type
void schwarz_apply(const MeshData& m, const SchwarzData& sw, sem_dtype t, const void* r, void* z, void* tmp_ovl,
                   hipStream_t s);
void chebyshev_coefficients(PmgLevel& lv, double lo, double hi, int degree);
}  // namespace sem

struct sem_pmg_s {
  sem_mesh base = nullptr;
  sem_pmg_opts o{};
  int n_levels = 0;
  int orders[sem::kMaxLevels] = {0};
  std::vector<sem::PmgLevel> lv;
  std::vector<sem_mesh_s*> owned;   // coarse level meshes (deleted with the hierarchy)
  ~sem_pmg_s() {
    for (sem_mesh_s* m : owned) delete m;
  }
};
