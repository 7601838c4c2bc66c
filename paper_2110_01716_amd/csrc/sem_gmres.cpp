// Flexible GMRES(K) outer solver (Implementation, FlexCG/GMRES paragraph;
// Performance Results, the GMRES trial with K bounded by 6).
//
// Right-preconditioned flexible GMRES (Saad 1993): the preconditioner may
// change from one application to the next (the pMG V-cycle with an inexact
// coarse solve does), so the preconditioned directions z_j = M(v_j) are kept
// alongside the Arnoldi basis v_j, and the update is x += Z y. Each Arnoldi
// step orthogonalises w = A z_j against v_0..v_j by one round of classical
// Gram-Schmidt, with the coefficients h_ij = (v_i, w) and (w, w) taken by a
// single multi-dot; the new norm comes from Pythagoras,
// |w - V h|^2 = (w, w) - |h|^2, unless cancellation makes that inaccurate
// (then it is recomputed from the vector). Givens rotations on the host
// keep the least-squares residual |g_{j+1}| = |b - A x_j| in exact arithmetic,
// which is the convergence test. After K steps without convergence the method
// restarts from the true residual.
//
// Storage (FP64 E-vectors): K + 1 basis vectors and K preconditioned
// directions. A w = A z_j is written straight into v_{j+1}'s slot and
// orthogonalised in place.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <vector>

#include "sem_internal.h"

using namespace sem;

namespace {

struct Pooled {
  void* p = nullptr;
  size_t bytes = 0;
  Pooled() = default;
  Pooled(const Pooled&) = delete;
  Pooled& operator=(const Pooled&) = delete;
  ~Pooled() { pool_put(p, bytes); }
  void get(size_t n) {
    bytes = n;
    p = pool_get(n);
  }
};

}  // namespace

extern "C" int sem_gmres_solve(sem_mesh m, sem_pmg pm, int K, const double* b, double* x, const sem_solve_opts* oin,
                               sem_solve_info* info, void* stream) {
  int rc = SEM_OK;
  const int g = guarded([&] {
    const auto t0 = std::chrono::steady_clock::now();
    if (!m || !b || !x) fail(SEM_EINVAL, "sem_gmres_solve: NULL argument");
    if (K < 1 || K > 64) fail(SEM_EINVAL, "sem_gmres_solve: K=%d outside [1,64]", K);
    if (pm && pm->base != m) fail(SEM_EINVAL, "sem_gmres_solve: pMG hierarchy of another mesh");
    sem_solve_opts o;
    sem_solve_opts_default(&o);
    if (oin) o = *oin;
    if (o.lambda != 0.0 && pm) fail(SEM_EINVAL, "sem_gmres_solve: Helmholtz solves use the Jacobi preconditioner");
    if (o.lambda < 0.0 || !std::isfinite(o.lambda)) fail(SEM_EINVAL, "sem_gmres_solve: lambda must be >= 0");
    if (o.maxit < 1 && o.fixed_iters < 1) fail(SEM_EINVAL, "sem_gmres_solve: maxit must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    const MeshData& md = m->d;
    const int64_t n = md.nloc;
    const size_t vb = (sizeof(double) * n + 255) & ~size_t(255);
    const int64_t stride = vec_blocks(n);
    const double lam = o.lambda;

    // workspace: V[K+1], Z[K], dinv (Helmholtz), partial [(K+2) x stride], small device arrays
    Pooled ws;
    const size_t sa = (sizeof(double) * (K + 2) + 255) & ~size_t(255);  // one small device array
    const size_t small = 4 * sa;
    ws.get(vb * (2 * K + 2) + sizeof(double) * stride * (K + 2) + small);
    uint8_t* base = static_cast<uint8_t*>(ws.p);
    std::vector<double*> V(K + 1), Z(K);
    for (int i = 0; i <= K; ++i) V[i] = reinterpret_cast<double*>(base + vb * i);
    for (int i = 0; i < K; ++i) Z[i] = reinterpret_cast<double*>(base + vb * (K + 1 + i));
    double* dinv_h = reinterpret_cast<double*>(base + vb * (2 * K + 1));
    double* partial = reinterpret_cast<double*>(base + vb * (2 * K + 2));
    uint8_t* sm = reinterpret_cast<uint8_t*>(partial + stride * (K + 2));
    const double** ptrV = reinterpret_cast<const double**>(sm);           // K+1 pointers
    const double** ptrZ = reinterpret_cast<const double**>(sm + sa);      // K pointers
    double* dcoef = reinterpret_cast<double*>(sm + 2 * sa);               // K+1 coefficients
    double* dout = reinterpret_cast<double*>(sm + 3 * sa);                // multi-dot results, K+2
    SEM_HIP(hipMemcpyAsync(ptrV, V.data(), sizeof(double*) * (K + 1), hipMemcpyHostToDevice, s));
    SEM_HIP(hipMemcpyAsync(ptrZ, Z.data(), sizeof(double*) * K, hipMemcpyHostToDevice, s));
    SEM_HIP(hipStreamSynchronize(s));

    const double* dinv = md.dinv64.as<double>();
    if (lam != 0.0) {
      helmholtz_dinv(md, lam, dinv_h, V[0], s);
      dinv = dinv_h;
    }
    std::unique_ptr<VcycleRunner, void (*)(VcycleRunner*)> vc(pm ? vcycle_runner_create(pm, s) : nullptr,
                                                              vcycle_runner_destroy);
    auto apply_op = [&](const double* u, double* out) {
      if (lam != 0.0) apply_H(md, lam, u, out, s);
      else apply_A(md, SEM_F64, u, out, s);
    };
    auto precond = [&](const double* r, double* z) {
      if (vc) vcycle_runner_apply(vc.get(), r, z);
      else vec_op1(V_SCALE_DINV, n, z, r, 0.0, dinv, s);
    };

    sem_solve_info inf{};
    inf.relres_initial = 1.0;
    SEM_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    const double bb = mesh_dot_ws(md, b, b, partial, s);
    if (!std::isfinite(bb)) {
      inf.status = SEM_ENAN;
      rc = SEM_ENAN;
      set_error("sem_gmres_solve: NaN or Inf in the right-hand side");
    } else if (bb == 0.0) {
      inf.status = SEM_OK;
    } else {
      const double bnorm = std::sqrt(bb);
      const bool fixed = o.fixed_iters > 0;
      const int64_t limit = fixed ? o.fixed_iters : o.maxit;
      std::vector<double> H((size_t)(K + 1) * K), cs(K), sn(K), gv(K + 1), h(K + 2), y(K);
      auto Hc = [&](int i, int j) -> double& { return H[(size_t)j * (K + 1) + i]; };
      double beta = bnorm;
      vec_op1(V_SCALE, n, V[0], b, 1.0 / beta, nullptr, s);
      int64_t iters = 0;
      bool done = false;
      int status = SEM_OK;
      double resid = beta;
      while (!done) {
        std::fill(gv.begin(), gv.end(), 0.0);
        gv[0] = beta;
        int j = 0;
        for (; j < K; ++j) {
          precond(V[j], Z[j]);
          apply_op(Z[j], V[j + 1]);
          // h_ij = (v_i, w), i <= j, and (w, w): one multi-dot over slots 0..j+1
          mesh_multidot(md, ptrV, j + 2, V[j + 1], partial, stride, dout, s);
          SEM_HIP(hipMemcpyAsync(h.data(), dout, sizeof(double) * (j + 2), hipMemcpyDeviceToHost, s));
          SEM_HIP(hipStreamSynchronize(s));
          const double ww = h[j + 1];
          double g2 = ww;
          for (int i = 0; i <= j; ++i) g2 -= h[i] * h[i];
          bool finite = std::isfinite(g2);
          for (int i = 0; i <= j; ++i) finite = finite && std::isfinite(h[i]);
          if (!finite) {
            status = SEM_ENAN;
            done = true;
            break;
          }
          SEM_HIP(hipMemcpyAsync(dcoef, h.data(), sizeof(double) * (j + 1), hipMemcpyHostToDevice, s));
          double gam;
          if (g2 > 1e-6 * ww) {
            gam = std::sqrt(g2);
            mesh_lincomb(md, ptrV, j + 1, dcoef, V[j + 1], 1.0, -1.0, 1.0 / gam, V[j + 1], s);
          } else {
            // cancellation: orthogonalise, then take the norm from the vector
            mesh_lincomb(md, ptrV, j + 1, dcoef, V[j + 1], 1.0, -1.0, 1.0, V[j + 1], s);
            gam = std::sqrt(std::max(mesh_dot_ws(md, V[j + 1], V[j + 1], partial, s), 0.0));
            if (gam > 0.0) vec_op1(V_SCALE, n, V[j + 1], V[j + 1], 1.0 / gam, nullptr, s);
          }
          SEM_HIP(hipStreamSynchronize(s));  // h is reused next step
          for (int i = 0; i <= j; ++i) Hc(i, j) = h[i];
          Hc(j + 1, j) = gam;
          // previous rotations, then a new one that zeroes H(j+1, j)
          for (int i = 0; i < j; ++i) {
            const double a = Hc(i, j), c = Hc(i + 1, j);
            Hc(i, j) = cs[i] * a + sn[i] * c;
            Hc(i + 1, j) = -sn[i] * a + cs[i] * c;
          }
          const double a = Hc(j, j), c = Hc(j + 1, j);
          const double r = std::hypot(a, c);
          cs[j] = r > 0 ? a / r : 1.0;
          sn[j] = r > 0 ? c / r : 0.0;
          Hc(j, j) = r;
          Hc(j + 1, j) = 0.0;
          gv[j + 1] = -sn[j] * gv[j];
          gv[j] = cs[j] * gv[j];
          resid = std::fabs(gv[j + 1]);
          ++iters;
          const bool breakdown = !(gam > 1e-14 * std::sqrt(ww));
          if (fixed ? iters >= limit : (resid <= o.rtol * bnorm || iters >= limit)) {
            done = true;
            ++j;
            break;
          }
          if (breakdown) {  // the Krylov space is invariant: the update below is exact
            done = true;
            ++j;
            break;
          }
        }
        if (status == SEM_ENAN) break;
        // y = H(0:j, 0:j)^-1 g(0:j), then x += Z y
        const int k = std::min(j, K);
        for (int i = k - 1; i >= 0; --i) {
          double t = gv[i];
          for (int l = i + 1; l < k; ++l) t -= Hc(i, l) * y[l];
          y[i] = t / Hc(i, i);
        }
        SEM_HIP(hipMemcpyAsync(dcoef, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
        mesh_lincomb(md, ptrZ, k, dcoef, x, 1.0, 1.0, 1.0, x, s);
        SEM_HIP(hipStreamSynchronize(s));
        if (done) break;
        // restart from the true residual: v_0 = (b - A x) / |b - A x|
        apply_op(x, V[0]);
        vec_op1(V_SCALE, n, V[0], V[0], -1.0, nullptr, s);
        vec_op1(V_AXPY, n, V[0], b, 1.0, nullptr, s);
        beta = std::sqrt(std::max(mesh_dot_ws(md, V[0], V[0], partial, s), 0.0));
        if (!std::isfinite(beta)) {
          status = SEM_ENAN;
          break;
        }
        if (beta == 0.0) break;
        vec_op1(V_SCALE, n, V[0], V[0], 1.0 / beta, nullptr, s);
      }
      if (status == SEM_OK && !fixed && resid > o.rtol * bnorm) status = SEM_ENOCONV;
      inf.iters = (int32_t)iters;
      inf.status = status;
      inf.relres = resid / bnorm;
      // true residual at exit
      apply_op(x, V[0]);
      vec_op1(V_SCALE, n, V[0], V[0], -1.0, nullptr, s);
      vec_op1(V_AXPY, n, V[0], b, 1.0, nullptr, s);
      inf.relres_true = std::sqrt(std::max(mesh_dot_ws(md, V[0], V[0], partial, s), 0.0)) / bnorm;
      if (vc) inf.coarse_iters = vcycle_runner_coarse_iters(vc.get());
      rc = status;
      if (status == SEM_ENOCONV) set_error("sem_gmres_solve: iteration limit reached");
      if (status == SEM_ENAN) set_error("sem_gmres_solve: NaN or Inf in an iterate");
    }
    SEM_HIP(hipStreamSynchronize(s));
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
  });
  return g != SEM_OK ? g : rc;
}
